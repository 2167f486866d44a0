// Host runtime of the stitching path: argument validation, the rig plan (the paper's
// start-up pre-allocation, Sec. 4.3.2), workspace layout, descriptor tables and the
// kernel launches.  Every host-checkable error is reported before anything is
// enqueued.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "stitch.h"
#include "stitch_internal.h"

using namespace stitch;

namespace {
thread_local std::string t_err = "";
}  // namespace

namespace stitch {
stitch_status fail(stitch_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  t_err = buf;
  return s;
}

stitch_status hip_fail(hipError_t e, const char* what) {
  return fail(STITCH_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}
}  // namespace stitch

namespace {

int64_t floor_div(int64_t a, int64_t b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }
int64_t ceil_div(int64_t a, int64_t b) { return -floor_div(-a, b); }
int64_t align_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

struct Rect {
  int x = 0, y = 0, w = 0, h = 0;
  bool empty() const { return w <= 0 || h <= 0; }
};

Rect intersect(const Rect& a, const Rect& b) {
  Rect r;
  r.x = std::max(a.x, b.x);
  r.y = std::max(a.y, b.y);
  r.w = std::min(a.x + a.w, b.x + b.w) - r.x;
  r.h = std::min(a.y + a.h, b.y + b.h) - r.y;
  if (r.w <= 0 || r.h <= 0) r = Rect{};
  return r;
}

int elem_size(int dtype) { return dtype == STITCH_F32 ? 4 : dtype == STITCH_F16 ? 2 : 1; }

}  // namespace

// Canvas -> source map: adj(H) / adj(H)[2][2] in FP64, cofactors formed as a*b - c*d,
// each entry rounded to FP32.  Returns false (with a reason) if H is unusable.
bool stitch::hinv_spec(const double* a, float out[9], double* sign_out, const char** why) {
#pragma clang fp contract(off)
  for (int i = 0; i < 9; ++i)
    if (!std::isfinite(a[i])) { *why = "homography has a non-finite entry"; return false; }
  double adj[9];
  adj[0] = a[4] * a[8] - a[5] * a[7];
  adj[1] = a[2] * a[7] - a[1] * a[8];
  adj[2] = a[1] * a[5] - a[2] * a[4];
  adj[3] = a[5] * a[6] - a[3] * a[8];
  adj[4] = a[0] * a[8] - a[2] * a[6];
  adj[5] = a[2] * a[3] - a[0] * a[5];
  adj[6] = a[3] * a[7] - a[4] * a[6];
  adj[7] = a[1] * a[6] - a[0] * a[7];
  adj[8] = a[0] * a[4] - a[1] * a[3];
  for (int i = 0; i < 9; ++i)
    if (!std::isfinite(adj[i])) { *why = "adjugate of H is not finite"; return false; }
  if (adj[8] == 0.0) { *why = "adj(H)[2][2] == 0: the inverse cannot be normalised"; return false; }
  for (int i = 0; i < 9; ++i) {
    const double q = adj[i] / adj[8];
    const float f = (float)q;
    if (!std::isfinite(q) || !std::isfinite(f)) { *why = "normalised inverse overflows FP32"; return false; }
    out[i] = f;
  }
  if (sign_out) {
    // det(H) = sum_j H[0][j] adj[j][0]; z at the canvas side has the sign of
    // (source-side w) * det / adj22.
    const double det = a[0] * adj[0] + a[1] * adj[3] + a[2] * adj[6];
    *sign_out = (det / adj[8]) > 0.0 ? 1.0 : -1.0;
  }
  return true;
}

namespace {

// Canvas bounding box of the pixels the warp can make non-zero (inclusive), or false
// when the footprint is unbounded (part of the source lies beyond the horizon).
bool footprint_bbox(const double* H, double sign, int fw, int fh, int64_t bb[4]) {
  const double xs[4] = {-1.0, (double)fw, (double)fw, -1.0};
  const double ys[4] = {-1.0, -1.0, (double)fh, (double)fh};
  double x0 = 1e300, x1 = -1e300, y0 = 1e300, y1 = -1e300;
  for (int i = 0; i < 4; ++i) {
    const double w = H[6] * xs[i] + H[7] * ys[i] + H[8];
    if (!(w * sign > 0.0)) return false;
    const double X = (H[0] * xs[i] + H[1] * ys[i] + H[2]) / w;
    const double Y = (H[3] * xs[i] + H[4] * ys[i] + H[5]) / w;
    if (!std::isfinite(X) || !std::isfinite(Y) || std::fabs(X) > 1e9 || std::fabs(Y) > 1e9) return false;
    x0 = std::min(x0, X); x1 = std::max(x1, X);
    y0 = std::min(y0, Y); y1 = std::max(y1, Y);
  }
  // two pixels of slack for the FP32 coordinate arithmetic
  bb[0] = (int64_t)std::floor(x0) - 2;
  bb[1] = (int64_t)std::ceil(x1) + 2;
  bb[2] = (int64_t)std::floor(y0) - 2;
  bb[3] = (int64_t)std::ceil(y1) + 2;
  return true;
}

struct Interval { int64_t a, b; };   // inclusive, a > b means empty

// Support of REDUCE(g) given the support of g (non-negative weights cannot cancel).
Interval reduce_support(Interval s) { return {ceil_div(s.a - 2, 2), floor_div(s.b + 2, 2)}; }

// Per-launch HIP-event timing (diagnostics).  While enabled, a call records one event on
// its stream before its first launch and one after every launch; the time between two
// consecutive events is charged to the launch's kind.
struct EventLog {
  static constexpr int kKinds = 2 * kMaxLevels;
  bool on = false;
  std::vector<hipEvent_t> spare;
  struct Call { std::vector<hipEvent_t> ev; std::vector<int> kind; };   // ev[i] .. ev[i+1] = launch i
  std::vector<Call> done;
  Call cur;
  double ms[kKinds] = {};
  int32_t n[kKinds] = {};

  ~EventLog() {
    recycle();
    for (hipEvent_t e : spare) (void)hipEventDestroy(e);
  }
  void recycle() {
    for (auto& c : done)
      for (hipEvent_t e : c.ev) spare.push_back(e);
    done.clear();
    for (hipEvent_t e : cur.ev) spare.push_back(e);
    cur = Call();
  }
  void reset(bool enable) {
    on = enable;
    recycle();
    for (int i = 0; i < kKinds; ++i) { ms[i] = 0.0; n[i] = 0; }
  }
  // kind < 0: the event before a call's first launch
  stitch_status mark(hipStream_t s, int kind) {
    if (!on) return STITCH_OK;
    hipEvent_t ev;
    if (!spare.empty()) {
      ev = spare.back();
      spare.pop_back();
    } else {
      const hipError_t ce = hipEventCreate(&ev);
      if (ce != hipSuccess) return hip_fail(ce, "timing event create");
    }
    const hipError_t re = hipEventRecord(ev, s);
    if (re != hipSuccess) { spare.push_back(ev); return hip_fail(re, "timing event record"); }
    cur.ev.push_back(ev);
    if (kind >= 0) cur.kind.push_back(kind);
    return STITCH_OK;
  }
  // end of a call: keep its events if they are complete, else give them back
  void end_call() {
    if (!cur.ev.empty() && cur.kind.size() + 1 == cur.ev.size()) done.push_back(std::move(cur));
    else
      for (hipEvent_t e : cur.ev) spare.push_back(e);
    cur = Call();
  }
  // wait for the recorded events and add their intervals to the totals
  stitch_status collect() {
    stitch_status st = STITCH_OK;
    for (auto& c : done) {
      if (!st) {
        const hipError_t e = hipEventSynchronize(c.ev.back());
        if (e != hipSuccess) st = hip_fail(e, "timing event synchronise");
      }
      for (size_t i = 0; !st && i < c.kind.size(); ++i) {
        float t = 0.0f;
        const hipError_t e = hipEventElapsedTime(&t, c.ev[i], c.ev[i + 1]);
        if (e != hipSuccess) { st = hip_fail(e, "timing elapsed"); break; }
        ms[c.kind[i]] += t;
        n[c.kind[i]] += 1;
      }
      for (hipEvent_t e : c.ev) spare.push_back(e);
    }
    done.clear();
    return st;
  }
};

struct CamPlan {
  int fw = 0, fh = 0;
  float hinv[9] = {};
  Rect roi[kMaxLevels];
  Rect band[kMaxLevels];
  // where L_k is stored and read: the band window widened to 8-sample column boundaries
  // (inside roi), so band rows go out as whole 16-byte vectors at either storage size; the
  // added columns carry seam weight 0
  Rect lwin[kMaxLevels];
  std::vector<uint8_t> mask0;     // seam weights on roi[0], rows of mask_row bytes
  // the seam weights on their own support box (for the float-frame forward and its
  // vector-Jacobian product, which define every array on the whole canvas)
  std::vector<uint8_t> wsup;
  int wsx = 0, wsy = 0, wsw = 0, wsh = 0;
  int64_t mask_row = 0;
  size_t off_mask0 = 0;
  size_t off_g[kMaxLevels] = {};  int64_t g_row[kMaxLevels] = {}, g_plane[kMaxLevels] = {};
  size_t off_gm[kMaxLevels] = {}; int64_t gm_row[kMaxLevels] = {};
  size_t off_l[kMaxLevels] = {};  int64_t l_row[kMaxLevels] = {}, l_plane[kMaxLevels] = {};
};

}  // namespace

struct stitch_plan {
  int n = 0, W = 0, H = 0, L = 0, storage = STITCH_F32, flags = 0, es = 4;
  int dw[kMaxLevels] = {}, dh[kMaxLevels] = {};
  std::vector<CamPlan> cam;
  size_t off_r[kMaxLevels] = {};
  int64_t r_row[kMaxLevels] = {}, r_plane[kMaxLevels] = {};
  bool has_r[kMaxLevels] = {};
  // descriptor tables: pyramid passes k = 0..L-2, blend levels k = 0..L-1
  std::vector<PyrItem> items[kMaxLevels];
  int tiles[kMaxLevels] = {};
  size_t off_items[kMaxLevels] = {};
  // pyramid-pass settings: requested tile sub-steps (0: the planner's choice), the ones in
  // use, and persistent workgroups per compute unit (0: as many as fit, -1: one per tile)
  int sub_req[kMaxLevels] = {};
  int sub[kMaxLevels] = {};
  int wg_cap[kMaxLevels] = {};
  std::vector<BlendCam> bcams[kMaxLevels];
  size_t off_bcams[kMaxLevels] = {};
  std::vector<BlendItem> bitems;            // one per level
  size_t off_bitems = 0;
  size_t ws_bytes = 0;
  uint8_t* ws = nullptr;
  EventLog timing;   // optional per-launch event timing (diagnostics)
};

int stitch::plan_levels(const stitch_plan* p) { return p->L; }

void stitch::plan_camera(const stitch_plan* p, int i, PlanCamera* out) {
  const CamPlan& c = p->cam[i];
  out->fw = c.fw;
  out->fh = c.fh;
  for (int j = 0; j < 9; ++j) out->hinv[j] = c.hinv[j];
  out->wx = c.wsx; out->wy = c.wsy; out->ww = c.wsw; out->wh = c.wsh;
  out->weights = c.wsup.empty() ? nullptr : c.wsup.data();
}

void stitch::plan_geometry(const stitch_plan* p, int* n, int* frame_w, int* frame_h, int* canvas_w, int* canvas_h,
                           bool* bound) {
  *n = p->n;
  for (int i = 0; i < p->n; ++i) {
    frame_w[i] = p->cam[i].fw;
    frame_h[i] = p->cam[i].fh;
  }
  *canvas_w = p->W;
  *canvas_h = p->H;
  *bound = p->ws != nullptr;
}

namespace {

// Bump allocator over the workspace (offsets only, 256-byte aligned).
struct Layout {
  size_t top = 0;
  size_t take(size_t bytes) {
    const size_t off = top;
    top = (size_t)align_up((int64_t)(top + bytes), 256);
    return off;
  }
};

int64_t row_elems(int w, int es) { return align_up((int64_t)w * es, 256) / es; }

}  // namespace

// Validate a caller image view.
stitch_status stitch::check_image(const stitch_image* im, const char* name, int dtype, int layout, int channels) {
  if (!im) return fail(STITCH_E_NULL, "%s is NULL", name);
  if (!im->data) return fail(STITCH_E_NULL, "%s->data is NULL", name);
  if (im->width <= 0 || im->height <= 0)
    return fail(STITCH_E_SHAPE, "%s has non-positive size %dx%d", name, im->width, im->height);
  if (dtype >= 0 && im->dtype != dtype) return fail(STITCH_E_SHAPE, "%s has dtype %d, expected %d", name, im->dtype, dtype);
  if (layout >= 0 && im->layout != layout)
    return fail(STITCH_E_SHAPE, "%s has layout %d, expected %d", name, im->layout, layout);
  if (channels > 0 && im->channels != channels)
    return fail(STITCH_E_SHAPE, "%s has %d channels, expected %d", name, im->channels, channels);
  const int es = elem_size(im->dtype);
  if (im->dtype != STITCH_U8 && im->dtype != STITCH_F16 && im->dtype != STITCH_F32)
    return fail(STITCH_E_UNSUPPORTED, "%s has unknown dtype %d", name, im->dtype);
  if (im->layout == STITCH_HWC) {
    if (im->row_pitch < (int64_t)im->width * im->channels * es)
      return fail(STITCH_E_SHAPE, "%s row pitch %lld too small", name, (long long)im->row_pitch);
  } else if (im->layout == STITCH_CHW) {
    if (im->row_pitch < (int64_t)im->width * es || im->row_pitch % es)
      return fail(STITCH_E_SHAPE, "%s row pitch %lld invalid", name, (long long)im->row_pitch);
    if (im->channels > 1 && (im->plane_pitch < im->row_pitch * im->height || im->plane_pitch % es))
      return fail(STITCH_E_SHAPE, "%s plane pitch %lld invalid", name, (long long)im->plane_pitch);
  } else {
    return fail(STITCH_E_SHAPE, "%s has unknown layout %d", name, im->layout);
  }
  return STITCH_OK;
}

namespace {

stitch_status check_levels_dims(int W, int H, int L, int dw[], int dh[]) {
  if (L < 1 || L > kMaxLevels) return fail(STITCH_E_LEVELS, "levels %d outside 1..%d", L, kMaxLevels);
  if (W <= 0 || H <= 0) return fail(STITCH_E_SHAPE, "canvas %dx%d is empty", W, H);
  dw[0] = W;
  dh[0] = H;
  for (int k = 1; k < L; ++k) {
    dw[k] = (dw[k - 1] + 1) / 2;
    dh[k] = (dh[k - 1] + 1) / 2;
  }
  for (int k = 0; k < L; ++k)
    if (dw[k] < 3 || dh[k] < 3)
      return fail(STITCH_E_LEVELS, "level %d of a %dx%d canvas is %dx%d; every side must be >= 3", k, W, H, dw[k],
                  dh[k]);
  return STITCH_OK;
}

stitch_status upload(void* dst, const void* src, size_t bytes, hipStream_t s, const char* what) {
  if (bytes == 0) return STITCH_OK;
  const hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
  return e == hipSuccess ? STITCH_OK : hip_fail(e, what);
}

// Sub-steps per pyramid tile (tile height 16 * sub) for a launch of t16 16-row tiles: the
// tallest (fewest staged halo rows) that still leaves about eight tiles per compute unit.
// The pyramid pass addresses a level with 32-bit element offsets and 24-bit row products:
// every plane set must span fewer than 2^31 elements and every row fewer than 2^23.
bool fits_offsets(int64_t row, int64_t plane, int64_t rows, int nplanes) {
  return row < ((int64_t)1 << 23) && (int64_t)(nplanes - 1) * plane + rows * row < ((int64_t)1 << 31);
}

int choose_sub(int64_t t16) {
  for (int sub = 8; sub > 1; sub >>= 1)
    if (t16 / sub >= 2048) return sub;
  return 1;
}

void set_sub(std::vector<PyrItem>& items, int sub, int& tiles) {
  tiles = 0;
  for (PyrItem& it : items) {
    it.sub = sub;
    it.tiles_y = (it.rows16 + sub - 1) / sub;
    it.tile_begin = tiles;
    tiles += it.tiles_x * it.tiles_y;
  }
}

// Fill the pyramid-pass and blend tables of a plan whose workspace base is ws.
void build_tables(stitch_plan* p) {
  uint8_t* ws = p->ws;
  const int L = p->L;
  for (int k = 0; k + 1 < L; ++k) {
    p->items[k].clear();
    int tiles = 0;
    for (int i = 0; i < p->n; ++i) {
      const CamPlan& c = p->cam[i];
      const Rect r = c.roi[k];
      if (r.empty()) continue;
      PyrItem it;
      std::memset(&it, 0, sizeof it);
      it.tile_begin = tiles;
      it.tiles_x = (r.w + kPyrTX - 1) / kPyrTX;
      it.rows16 = (r.h + kPyrTY - 1) / kPyrTY;
      it.sub = 1;
      it.tiles_y = it.rows16;
      it.tile_x0 = r.x;
      it.tile_y0 = r.y;
      it.fine_w = p->dw[k];
      it.fine_h = p->dh[k];
      it.roi_x = r.x; it.roi_y = r.y; it.roi_w = r.w; it.roi_h = r.h;
      it.nch = 3;
      if (k == 0) {
        it.img_kind = kSrcWarp;
        it.frame_slot = i;
        it.frame_w = c.fw;
        it.frame_h = c.fh;
        std::memcpy(it.hinv, c.hinv, sizeof it.hinv);
        it.msk_kind = kSrcU8;
        it.msk = ws + c.off_mask0;
        it.msk_row = c.mask_row;
      } else {
        it.img_kind = kSrcPlanes;
        it.img = ws + c.off_g[k];
        it.img_row = c.g_row[k];
        it.img_plane = c.g_plane[k];
        it.msk_kind = kSrcPlanes;
        it.msk = ws + c.off_gm[k];
        it.msk_row = c.gm_row[k];
      }
      const Rect cr = c.roi[k + 1];
      it.croi_x = cr.x; it.croi_y = cr.y; it.croi_w = cr.w; it.croi_h = cr.h;
      it.g_out = ws + c.off_g[k + 1];
      it.g_row = c.g_row[k + 1];
      it.g_plane = c.g_plane[k + 1];
      it.gm_out = ws + c.off_gm[k + 1];
      it.gm_row = c.gm_row[k + 1];
      const Rect b = c.lwin[k];
      if (!b.empty()) {
        it.lw_x = b.x; it.lw_y = b.y; it.lw_w = b.w; it.lw_h = b.h;
        it.l_out = ws + c.off_l[k];
        it.l_row = c.l_row[k];
        it.l_plane = c.l_plane[k];
      }
      tiles += it.tiles_x * it.tiles_y;
      p->items[k].push_back(it);
    }
    p->sub[k] = p->sub_req[k] > 0 ? p->sub_req[k] : choose_sub(tiles);
    set_sub(p->items[k], p->sub[k], tiles);
    p->tiles[k] = tiles;
  }
  for (int k = 0; k < L; ++k) {
    p->bcams[k].clear();
    for (int i = 0; i < p->n; ++i) {
      const CamPlan& c = p->cam[i];
      const Rect b = c.lwin[k];
      if (b.empty()) continue;
      BlendCam bc;
      std::memset(&bc, 0, sizeof bc);
      bc.lx = b.x; bc.ly = b.y; bc.lw = b.w; bc.lh = b.h;
      if (k + 1 < L) {
        bc.lap = ws + c.off_l[k];
        bc.lap_row = c.l_row[k];
        bc.lap_plane = c.l_plane[k];
      } else {   // top band = G_{L-1} (or G_0 stored by the warp when L == 1), viewed on the band window
        const Rect r = c.roi[k];
        bc.lap = ws + c.off_g[k] + ((int64_t)(b.y - r.y) * c.g_row[k] + (b.x - r.x)) * p->es;
        bc.lap_row = c.g_row[k];
        bc.lap_plane = c.g_plane[k];
      }
      const Rect r = c.roi[k];
      bc.wx = r.x; bc.wy = r.y; bc.ww = r.w; bc.wh = r.h;
      if (k == 0) {
        bc.wgt = ws + c.off_mask0;
        bc.wgt_row = c.mask_row;
        bc.wgt_u8 = 1;
      } else {
        bc.wgt = ws + c.off_gm[k];
        bc.wgt_row = c.gm_row[k];
      }
      p->bcams[k].push_back(bc);
    }
  }
  p->bitems.assign(L, BlendItem{});
  for (int k = 0; k < L; ++k) {
    BlendItem& bi = p->bitems[k];
    std::memset(&bi, 0, sizeof bi);
    bi.tiles_x = (p->dw[k] + kBlendTX - 1) / kBlendTX;
    bi.tiles_y = (p->dh[k] + kBlendTY - 1) / kBlendTY;
    bi.W = p->dw[k];
    bi.H = p->dh[k];
    bi.ncam = (int)p->bcams[k].size();
    bi.cams = (const BlendCam*)(ws + p->off_bcams[k]);
    if (k + 1 < L) {
      bi.has_coarse = 1;
      bi.cW = p->dw[k + 1];
      bi.cH = p->dh[k + 1];
      bi.r_in = ws + p->off_r[k + 1];
      bi.rin_row = p->r_row[k + 1];
      bi.rin_plane = p->r_plane[k + 1];
    }
    if (p->has_r[k]) {
      bi.r_out = ws + p->off_r[k];
      bi.rout_row = p->r_row[k];
      bi.rout_plane = p->r_plane[k];
    }
  }
}

// Check a frame set against the plan and collect its pointers for the level-0 pass.
stitch_status frame_args(const stitch_plan* p, const stitch_image* frames, FrameArgs& fa) {
  std::memset(&fa, 0, sizeof fa);
  fa.n = p->n;
  for (int i = 0; i < p->n; ++i) {
    char name[32];
    snprintf(name, sizeof name, "frames[%d]", i);
    const stitch_status st = check_image(&frames[i], name, STITCH_U8, STITCH_HWC, 3);
    if (st) return st;
    if (frames[i].width != p->cam[i].fw || frames[i].height != p->cam[i].fh)
      return fail(STITCH_E_SHAPE, "frames[%d] is %dx%d, planned %dx%d", i, frames[i].width, frames[i].height,
                  p->cam[i].fw, p->cam[i].fh);
    if (frames[i].row_pitch * (int64_t)frames[i].height >= ((int64_t)1 << 31) ||
        frames[i].row_pitch >= ((int64_t)1 << 24))
      return fail(STITCH_E_SHAPE, "frames[%d] spans 2 GiB or more, or its rows 16 MiB or more (offsets are "
                  "32-bit, row offsets 24-bit products)", i);
    fa.ptr[i] = (const uint8_t*)frames[i].data;
    fa.row[i] = frames[i].row_pitch;
  }
  return STITCH_OK;
}

}  // namespace

// ====================================================================================== API
extern "C" {

int32_t stitch_abi_version(void) { return STITCH_ABI_VERSION; }

const char* stitch_status_str(stitch_status s) {
  switch (s) {
    case STITCH_OK: return "ok";
    case STITCH_E_NULL: return "null pointer";
    case STITCH_E_SHAPE: return "inconsistent shape";
    case STITCH_E_LEVELS: return "invalid level count";
    case STITCH_E_HOMOGRAPHY: return "invalid homography";
    case STITCH_E_MASK: return "invalid seam weights";
    case STITCH_E_WORKSPACE: return "invalid workspace";
    case STITCH_E_DEVICE: return "device error";
    case STITCH_E_UNSUPPORTED: return "unsupported";
    case STITCH_E_STATE: return "invalid state";
  }
  return "unknown status";
}

const char* stitch_last_error(void) { return t_err.c_str(); }

// ------------------------------------------------------------------------------------ warp
stitch_status stitch_warp(const stitch_image* src, const double H[9], int32_t roi_x, int32_t roi_y,
                          stitch_image* dst, void* stream) {
  stitch_status st = check_image(src, "src", STITCH_U8, STITCH_HWC, 3);
  if (st) return st;
  if (!H) return fail(STITCH_E_NULL, "H is NULL");
  st = check_image(dst, "dst", -1, STITCH_CHW, 3);
  if (st) return st;
  if (dst->dtype != STITCH_F32 && dst->dtype != STITCH_F16)
    return fail(STITCH_E_UNSUPPORTED, "dst must be F32 or F16");
  float hi[9];
  const char* why = nullptr;
  if (!hinv_spec(H, hi, nullptr, &why)) return fail(STITCH_E_HOMOGRAPHY, "%s", why);
  const int es = elem_size(dst->dtype);
  const hipError_t e = launch_warp(dst->dtype == STITCH_F16, (const uint8_t*)src->data, src->row_pitch, src->width,
                                   src->height, hi, roi_x, roi_y, dst->data, dst->row_pitch / es,
                                   dst->plane_pitch / es, dst->width, dst->height, (hipStream_t)stream);
  return e == hipSuccess ? STITCH_OK : hip_fail(e, "warp launch");
}

stitch_status stitch_warp_coords(const double H[9], int32_t roi_x, int32_t roi_y, stitch_image* xy, void* stream) {
  if (!H) return fail(STITCH_E_NULL, "H is NULL");
  stitch_status st = check_image(xy, "xy", STITCH_F32, STITCH_CHW, 2);
  if (st) return st;
  float hi[9];
  const char* why = nullptr;
  if (!hinv_spec(H, hi, nullptr, &why)) return fail(STITCH_E_HOMOGRAPHY, "%s", why);
  const hipError_t e = launch_warp_coords(hi, roi_x, roi_y, (float*)xy->data, xy->row_pitch / 4, xy->plane_pitch / 4,
                                          xy->width, xy->height, (hipStream_t)stream);
  return e == hipSuccess ? STITCH_OK : hip_fail(e, "warp_coords launch");
}

// ------------------------------------------------------------------------------------ pyramid
size_t stitch_pyramid_workspace_bytes(int32_t levels) {
  return (size_t)align_up((int64_t)std::max(levels, 1) * (int64_t)sizeof(PyrItem), 256);
}

stitch_status stitch_pyramid(const stitch_image* g0, int32_t kind, stitch_levels* out, void* workspace,
                             size_t ws_bytes, void* stream) {
  if (!g0) return fail(STITCH_E_NULL, "g0 is NULL");
  if (!out) return fail(STITCH_E_NULL, "out is NULL");
  if (kind != 0 && kind != 1) return fail(STITCH_E_UNSUPPORTED, "kind must be 0 (Gaussian) or 1 (Laplacian)");
  const int L = out->levels;
  int dw[kMaxLevels], dh[kMaxLevels];
  stitch_status st = check_levels_dims(out->canvas_w, out->canvas_h, L, dw, dh);
  if (st) return st;
  const bool u8 = g0->dtype == STITCH_U8;
  st = check_image(g0, "g0", -1, u8 ? -1 : STITCH_CHW, -1);
  if (st) return st;
  if (u8 && g0->channels != 1) return fail(STITCH_E_SHAPE, "a U8 g0 must have one channel");
  if (!u8 && (g0->channels < 1 || g0->channels > 3))
    return fail(STITCH_E_UNSUPPORTED, "float g0 must have 1..3 channels");
  const int odt = out->level[0].dtype;
  if (odt != STITCH_F32 && odt != STITCH_F16) return fail(STITCH_E_UNSUPPORTED, "output levels must be F32 or F16");
  if (!u8 && g0->dtype != odt) return fail(STITCH_E_SHAPE, "float g0 and output levels must share a dtype");
  const int nch = g0->channels;
  for (int k = 0; k < L; ++k) {
    char name[32];
    snprintf(name, sizeof name, "out->level[%d]", k);
    st = check_image(&out->level[k], name, odt, STITCH_CHW, nch);
    if (st) return st;
    const Rect lr{out->origin_x[k], out->origin_y[k], out->level[k].width, out->level[k].height};
    if (lr.x < 0 || lr.y < 0 || lr.x + lr.w > dw[k] || lr.y + lr.h > dh[k])
      return fail(STITCH_E_SHAPE, "level %d rectangle leaves the %dx%d level canvas", k, dw[k], dh[k]);
    const int oes = elem_size(odt);
    if (!fits_offsets(out->level[k].row_pitch / oes, out->level[k].plane_pitch / oes, out->level[k].height, nch))
      return fail(STITCH_E_SHAPE, "%s spans 2^31 elements or more, or its rows 2^23 or more", name);
  }
  if (g0->width != out->level[0].width || g0->height != out->level[0].height)
    return fail(STITCH_E_SHAPE, "g0 and out->level[0] differ in size");
  if (L > 1 && (!workspace || ws_bytes < stitch_pyramid_workspace_bytes(L) || ((uintptr_t)workspace & 255)))
    return fail(STITCH_E_WORKSPACE, "workspace missing, misaligned or smaller than %zu bytes",
                stitch_pyramid_workspace_bytes(L));
  const hipStream_t s = (hipStream_t)stream;
  const bool f16 = odt == STITCH_F16;
  const int es = elem_size(odt);
  const stitch_image& l0 = out->level[0];
  hipError_t e = hipSuccess;
  if (g0->data != l0.data || u8) {
    e = launch_convert(f16, nch, u8, g0->data, g0->row_pitch / elem_size(g0->dtype),
                       g0->plane_pitch / elem_size(g0->dtype), l0.data, l0.row_pitch / es, l0.plane_pitch / es,
                       l0.width, l0.height, s);
    if (e != hipSuccess) return hip_fail(e, "convert launch");
  }
  if (L == 1) return STITCH_OK;
  std::vector<PyrItem> items(L - 1);
  std::vector<int> tiles(L - 1);
  for (int k = 0; k + 1 < L; ++k) {
    const stitch_image& f = out->level[k];
    const stitch_image& c = out->level[k + 1];
    PyrItem it;
    std::memset(&it, 0, sizeof it);
    const int fx = out->origin_x[k], fy = out->origin_y[k];
    const int cx = out->origin_x[k + 1], cy = out->origin_y[k + 1];
    // tiles cover the level-k rectangle and every fine sample under the level-(k+1) rectangle
    const int x0 = std::min(fx, 2 * cx) & ~1, y0 = std::min(fy, 2 * cy) & ~1;
    const int x1 = std::max(fx + f.width, 2 * (cx + c.width)), y1 = std::max(fy + f.height, 2 * (cy + c.height));
    it.tiles_x = (x1 - x0 + kPyrTX - 1) / kPyrTX;
    it.tiles_y = (y1 - y0 + kPyrTY - 1) / kPyrTY;
    it.rows16 = it.tiles_y;
    it.sub = 1;
    it.tile_x0 = x0;
    it.tile_y0 = y0;
    it.fine_w = dw[k];
    it.fine_h = dh[k];
    it.roi_x = fx; it.roi_y = fy; it.roi_w = f.width; it.roi_h = f.height;
    it.img_kind = kSrcPlanes;
    it.nch = nch;
    it.img = f.data;
    it.img_row = f.row_pitch / es;
    it.img_plane = f.plane_pitch / es;
    it.msk_kind = kSrcNone;
    it.croi_x = cx; it.croi_y = cy; it.croi_w = c.width; it.croi_h = c.height;
    it.g_out = c.data;
    it.g_row = c.row_pitch / es;
    it.g_plane = c.plane_pitch / es;
    items[k] = it;
    tiles[k] = it.tiles_x * it.tiles_y;
  }
  st = upload(workspace, items.data(), items.size() * sizeof(PyrItem), s, "pyramid table upload");
  if (st) return st;
  FrameArgs fa;
  std::memset(&fa, 0, sizeof fa);
  const PyrItem* dev = (const PyrItem*)workspace;
  for (int k = 0; k + 1 < L; ++k) {
    e = launch_pyr(f16, false, false, dev + k, 1, tiles[k], fa, s);
    if (e != hipSuccess) return hip_fail(e, "pyramid launch");
  }
  if (kind == 1) {
    for (int k = 0; k + 1 < L; ++k) {
      const stitch_image& f = out->level[k];
      const stitch_image& c = out->level[k + 1];
      e = launch_expand_sub(f16, nch, f.data, f.row_pitch / es, f.plane_pitch / es, out->origin_x[k],
                            out->origin_y[k], f.width, f.height, c.data, c.row_pitch / es, c.plane_pitch / es,
                            out->origin_x[k + 1], out->origin_y[k + 1], c.width, c.height, dw[k], dh[k], s);
      if (e != hipSuccess) return hip_fail(e, "expand launch");
    }
  }
  return STITCH_OK;
}

// ------------------------------------------------------------------------------------ blend
size_t stitch_blend_workspace_bytes(int32_t n, int32_t levels) {
  const int64_t L = std::max(levels, 1);
  return (size_t)align_up(std::max(n, 1) * L * (int64_t)sizeof(BlendCam), 256) +
         (size_t)align_up(L * (int64_t)sizeof(BlendItem), 256);
}

stitch_status stitch_blend(int32_t n, const stitch_levels* bands, const stitch_levels* weights, stitch_image* pano,
                           stitch_levels* keep_r, void* workspace, size_t ws_bytes, void* stream) {
  if (n < 1 || n > kMaxCameras) return fail(STITCH_E_SHAPE, "n = %d outside 1..%d", n, kMaxCameras);
  if (!bands || !weights) return fail(STITCH_E_NULL, "bands or weights is NULL");
  stitch_status st = check_image(pano, "pano", STITCH_U8, STITCH_HWC, 3);
  if (st) return st;
  const int W = pano->width, H = pano->height, L = bands[0].levels;
  int dw[kMaxLevels], dh[kMaxLevels];
  st = check_levels_dims(W, H, L, dw, dh);
  if (st) return st;
  const int dt = bands[0].level[0].dtype;
  if (dt != STITCH_F32 && dt != STITCH_F16) return fail(STITCH_E_UNSUPPORTED, "bands must be F32 or F16");
  const int es = elem_size(dt);
  for (int i = 0; i < n; ++i) {
    if (bands[i].levels != L || weights[i].levels != L)
      return fail(STITCH_E_LEVELS, "pyramid %d has a different level count", i);
    if (bands[i].canvas_w != W || bands[i].canvas_h != H || weights[i].canvas_w != W || weights[i].canvas_h != H)
      return fail(STITCH_E_SHAPE, "pyramid %d is on a different canvas than the panorama", i);
    for (int k = 0; k < L; ++k) {
      char name[48];
      snprintf(name, sizeof name, "bands[%d].level[%d]", i, k);
      st = check_image(&bands[i].level[k], name, dt, STITCH_CHW, 3);
      if (st) return st;
      snprintf(name, sizeof name, "weights[%d].level[%d]", i, k);
      const stitch_image& w = weights[i].level[k];
      st = check_image(&w, name, -1, w.dtype == STITCH_U8 ? -1 : STITCH_CHW, 1);
      if (st) return st;
      if (w.dtype != STITCH_U8 && w.dtype != dt)
        return fail(STITCH_E_SHAPE, "%s must be U8 or the band dtype", name);
      const stitch_image& bl = bands[i].level[k];
      const int wes = elem_size(w.dtype);
      if (!fits_offsets(bl.row_pitch / es, bl.plane_pitch / es, bl.height, 3) ||
          !fits_offsets(w.row_pitch / wes, 0, w.height, 1))
        return fail(STITCH_E_SHAPE, "pyramid %d level %d spans 2^31 elements or more, or its rows 2^23 or more", i, k);
    }
  }
  if (L > 1 && !keep_r) return fail(STITCH_E_NULL, "keep_r is required when levels > 1 (it holds R_k)");
  if (keep_r) {
    if (keep_r->levels != L || keep_r->canvas_w != W || keep_r->canvas_h != H)
      return fail(STITCH_E_SHAPE, "keep_r does not match the panorama pyramid");
    for (int k = (keep_r->level[0].data ? 0 : 1); k < L; ++k) {
      char name[32];
      snprintf(name, sizeof name, "keep_r->level[%d]", k);
      st = check_image(&keep_r->level[k], name, dt, STITCH_CHW, 3);
      if (st) return st;
      if (keep_r->origin_x[k] || keep_r->origin_y[k] || keep_r->level[k].width != dw[k] ||
          keep_r->level[k].height != dh[k])
        return fail(STITCH_E_SHAPE, "%s must cover the whole level canvas", name);
    }
  }
  if (!workspace || ws_bytes < stitch_blend_workspace_bytes(n, L) || ((uintptr_t)workspace & 255))
    return fail(STITCH_E_WORKSPACE, "workspace missing, misaligned or smaller than %zu bytes",
                stitch_blend_workspace_bytes(n, L));
  std::vector<BlendCam> tab((size_t)n * L);
  for (int k = 0; k < L; ++k)
    for (int i = 0; i < n; ++i) {
      BlendCam& bc = tab[(size_t)k * n + i];
      std::memset(&bc, 0, sizeof bc);
      const stitch_image& b = bands[i].level[k];
      const stitch_image& w = weights[i].level[k];
      bc.lap = b.data;
      bc.lap_row = b.row_pitch / es;
      bc.lap_plane = b.plane_pitch / es;
      bc.lx = bands[i].origin_x[k]; bc.ly = bands[i].origin_y[k]; bc.lw = b.width; bc.lh = b.height;
      bc.wgt = w.data;
      bc.wgt_u8 = w.dtype == STITCH_U8;
      bc.wgt_row = w.row_pitch / elem_size(w.dtype);
      bc.wx = weights[i].origin_x[k]; bc.wy = weights[i].origin_y[k]; bc.ww = w.width; bc.wh = w.height;
    }
  const hipStream_t s = (hipStream_t)stream;
  const BlendCam* dev = (const BlendCam*)workspace;
  const size_t items_off = (size_t)align_up((int64_t)tab.size() * (int64_t)sizeof(BlendCam), 256);
  std::vector<BlendItem> items(L);
  for (int k = 0; k < L; ++k) {
    BlendItem& a = items[k];
    std::memset(&a, 0, sizeof a);
    a.W = dw[k]; a.H = dh[k];
    a.ncam = n;
    a.cams = dev + (size_t)k * n;
    if (k + 1 < L) {
      a.has_coarse = 1;
      a.cW = dw[k + 1]; a.cH = dh[k + 1];
      const stitch_image& r = keep_r->level[k + 1];
      a.r_in = r.data; a.rin_row = r.row_pitch / es; a.rin_plane = r.plane_pitch / es;
    }
    if (keep_r && keep_r->level[k].data) {
      const stitch_image& r = keep_r->level[k];
      a.r_out = r.data; a.rout_row = r.row_pitch / es; a.rout_plane = r.plane_pitch / es;
    }
    if (k == 0) { a.pano = (uint8_t*)pano->data; a.pano_row = pano->row_pitch; }
    a.tiles_x = (dw[k] + kBlendTX - 1) / kBlendTX;
    a.tiles_y = (dh[k] + kBlendTY - 1) / kBlendTY;
  }
  st = upload(workspace, tab.data(), tab.size() * sizeof(BlendCam), s, "blend table upload");
  if (st) return st;
  st = upload((uint8_t*)workspace + items_off, items.data(), items.size() * sizeof(BlendItem), s, "blend table upload");
  if (st) return st;
  const BlendItem* idev = (const BlendItem*)((uint8_t*)workspace + items_off);
  for (int k = L - 1; k >= 0; --k) {
    const hipError_t e = launch_blend(dt == STITCH_F16, k == 0, idev + k, 1, items[k].tiles_x * items[k].tiles_y,
                                      PanoArg{nullptr, 0}, s, &items[k]);
    if (e != hipSuccess) return hip_fail(e, "blend launch");
  }
  return STITCH_OK;
}

// ------------------------------------------------------------------------------------ plan
stitch_status stitch_plan_create(int32_t n, const int32_t* frame_w, const int32_t* frame_h, const double* H,
                                 const uint8_t* const* masks, int32_t canvas_w, int32_t canvas_h, int32_t levels,
                                 int32_t storage, int32_t flags, stitch_plan** out) {
  if (!out) return fail(STITCH_E_NULL, "out is NULL");
  *out = nullptr;
  if (!frame_w || !frame_h || !H || !masks) return fail(STITCH_E_NULL, "frame_w, frame_h, H or masks is NULL");
  if (n < 1 || n > kMaxCameras) return fail(STITCH_E_SHAPE, "n = %d outside 1..%d", n, kMaxCameras);
  if (storage != STITCH_F32 && storage != STITCH_F16)
    return fail(STITCH_E_UNSUPPORTED, "storage must be STITCH_F32 or STITCH_F16");
  if (canvas_w > (1 << 20) || canvas_h > (1 << 20)) return fail(STITCH_E_SHAPE, "canvas side above 2^20");
  stitch_plan* p = new (std::nothrow) stitch_plan();
  if (!p) return fail(STITCH_E_UNSUPPORTED, "out of host memory");
  struct Guard { stitch_plan*& p; ~Guard() { delete p; } } guard{p};
  stitch_status st = check_levels_dims(canvas_w, canvas_h, levels, p->dw, p->dh);
  if (st) return st;
  p->n = n; p->W = canvas_w; p->H = canvas_h; p->L = levels;
  p->storage = storage; p->flags = flags; p->es = elem_size(storage);
  p->cam.resize(n);
  const int L = levels;
  // --- seam weights: present, partition of unity ---
  std::vector<uint16_t> total((size_t)canvas_w * canvas_h, 0);
  for (int i = 0; i < n; ++i) {
    if (!masks[i]) return fail(STITCH_E_NULL, "masks[%d] is NULL", i);
    const uint8_t* m = masks[i];
    for (size_t j = 0; j < total.size(); ++j) total[j] += m[j];
  }
  for (size_t j = 0; j < total.size(); ++j)
    if (total[j] != 255)
      return fail(STITCH_E_MASK, "seam weights sum to %d at canvas pixel (%zu, %zu); they must sum to 255",
                  (int)total[j], j % canvas_w, j / canvas_w);
  total.clear();
  total.shrink_to_fit();
  const int64_t A = (int64_t)1 << (L - 1);   // every ROI origin is a multiple of 2^(L-1)
  for (int i = 0; i < n; ++i) {
    CamPlan& c = p->cam[i];
    if (frame_w[i] < 3 || frame_h[i] <= 0 || frame_w[i] > (1 << 20) || frame_h[i] > (1 << 20))
      return fail(STITCH_E_SHAPE, "frame %d has size %dx%d (width 3 .. 2^20, height 1 .. 2^20)", i, frame_w[i],
                  frame_h[i]);
    c.fw = frame_w[i];
    c.fh = frame_h[i];
    const double* Hi = H + 9 * i;
    double sign = 1.0;
    const char* why = nullptr;
    if (!hinv_spec(Hi, c.hinv, &sign, &why)) return fail(STITCH_E_HOMOGRAPHY, "camera %d: %s", i, why);
    // --- where the warp can be non-zero, and what every level then needs ---
    int64_t bb[4];
    Rect roi0{0, 0, canvas_w, canvas_h};
    if (footprint_bbox(Hi, sign, c.fw, c.fh, bb)) {
      Interval sx{bb[0], bb[1]}, sy{bb[2], bb[3]};
      int64_t x0 = sx.a, x1 = sx.b, y0 = sy.a, y1 = sy.b;   // level-0 coordinates, inclusive
      // G_k support s_k; L_k support adds EXPAND(G_{k+1}); keep 3 samples of clearance
      // at every level (the seam-weight pyramid is exact only that far inside the ROI).
      Interval gx = sx, gy = sy;
      for (int k = 0; k < L; ++k) {
        Interval lx = gx, ly = gy;
        if (k + 1 < L) {
          const Interval nx = reduce_support(gx), ny = reduce_support(gy);
          lx = {std::min(gx.a, 2 * nx.a - 2), std::max(gx.b, 2 * nx.b + 2)};
          ly = {std::min(gy.a, 2 * ny.a - 2), std::max(gy.b, 2 * ny.b + 2)};
          x0 = std::min(x0, (lx.a - 3) * (int64_t(1) << k)); x1 = std::max(x1, (lx.b + 4) * (int64_t(1) << k) - 1);
          y0 = std::min(y0, (ly.a - 3) * (int64_t(1) << k)); y1 = std::max(y1, (ly.b + 4) * (int64_t(1) << k) - 1);
          gx = nx;
          gy = ny;
        } else {
          x0 = std::min(x0, (lx.a - 3) * (int64_t(1) << k)); x1 = std::max(x1, (lx.b + 4) * (int64_t(1) << k) - 1);
          y0 = std::min(y0, (ly.a - 3) * (int64_t(1) << k)); y1 = std::max(y1, (ly.b + 4) * (int64_t(1) << k) - 1);
        }
      }
      const int64_t rx0 = std::max<int64_t>(0, floor_div(x0, A) * A);
      const int64_t ry0 = std::max<int64_t>(0, floor_div(y0, A) * A);
      const int64_t rx1 = std::min<int64_t>(canvas_w, ceil_div(x1 + 1, A) * A);
      const int64_t ry1 = std::min<int64_t>(canvas_h, ceil_div(y1 + 1, A) * A);
      roi0 = (rx0 < rx1 && ry0 < ry1) ? Rect{(int)rx0, (int)ry0, (int)(rx1 - rx0), (int)(ry1 - ry0)} : Rect{};
    }
    for (int k = 0; k < L; ++k) {
      if (roi0.empty()) { c.roi[k] = Rect{}; continue; }
      const int xa = roi0.x >> k, ya = roi0.y >> k;
      const int xb = std::min<int>(p->dw[k], (int)ceil_div(roi0.x + roi0.w, (int64_t)1 << k));
      const int yb = std::min<int>(p->dh[k], (int)ceil_div(roi0.y + roi0.h, (int64_t)1 << k));
      c.roi[k] = Rect{xa, ya, xb - xa, yb - ya};
    }
    // --- seam-weight support per level (bounding box), and the band windows ---
    const uint8_t* m = masks[i];
    int64_t mx0 = canvas_w, mx1 = -1, my0 = canvas_h, my1 = -1;
    for (int y = 0; y < canvas_h; ++y) {
      const uint8_t* row = m + (size_t)y * canvas_w;
      for (int x = 0; x < canvas_w; ++x)
        if (row[x]) {
          mx0 = std::min<int64_t>(mx0, x); mx1 = std::max<int64_t>(mx1, x);
          my0 = std::min<int64_t>(my0, y); my1 = std::max<int64_t>(my1, y);
        }
    }
    if (mx1 >= mx0) {
      c.wsx = (int)mx0; c.wsy = (int)my0; c.wsw = (int)(mx1 - mx0 + 1); c.wsh = (int)(my1 - my0 + 1);
      c.wsup.resize((size_t)c.wsw * c.wsh);
      for (int y = 0; y < c.wsh; ++y)
        std::memcpy(&c.wsup[(size_t)y * c.wsw], m + (size_t)(c.wsy + y) * canvas_w + c.wsx, c.wsw);
    }
    Interval nx{mx0, mx1}, ny{my0, my1};
    for (int k = 0; k < L; ++k) {
      if (k > 0) { nx = reduce_support(nx); ny = reduce_support(ny); }
      Rect nk;
      if (nx.a <= nx.b && ny.a <= ny.b) {
        const int64_t xa = std::max<int64_t>(0, nx.a), xb = std::min<int64_t>(p->dw[k] - 1, nx.b);
        const int64_t ya = std::max<int64_t>(0, ny.a), yb = std::min<int64_t>(p->dh[k] - 1, ny.b);
        if (xa <= xb && ya <= yb) nk = Rect{(int)xa, (int)ya, (int)(xb - xa + 1), (int)(yb - ya + 1)};
      }
      c.band[k] = intersect(nk, c.roi[k]);
    }
    // --- shrink the ROIs to what the blend reads ---
    // The blend reads L_k on band_k only.  L_k there needs G_k on band_k and G_{k+1} on
    // EXPAND's support of band_k; G_k needs G_{k-1} on REDUCE's support; the weights Gm_k on
    // band_k need Gm_{k-1} on REDUCE's support down to the uint8 map.  Every such value is
    // computed from values inside these needed sets only, so an ROI that covers them (aligned
    // as before) keeps every value the blend reads exact; the rest of the footprint is skipped.
    if (!c.roi[0].empty()) {
      int64_t nx0 = INT64_MAX, nx1 = INT64_MIN, ny0 = INT64_MAX, ny1 = INT64_MIN;   // level-0 need, inclusive
      for (int ax = 0; ax < 2; ++ax) {
        Interval need[kMaxLevels], mneed[kMaxLevels];
        for (int k = 0; k < L; ++k) need[k] = mneed[k] = Interval{1, 0};
        auto band_iv = [&](int k) {
          const Rect b = c.band[k];
          if (b.empty()) return Interval{1, 0};
          return ax == 0 ? Interval{b.x, b.x + b.w - 1} : Interval{b.y, b.y + b.h - 1};
        };
        auto unite = [](Interval a, Interval b) {
          if (a.a > a.b) return b;
          if (b.a > b.b) return a;
          return Interval{std::min(a.a, b.a), std::max(a.b, b.b)};
        };
        auto rsup = [](Interval a) { return a.a > a.b ? a : Interval{2 * a.a - 2, 2 * a.b + 2}; };
        auto esup = [](Interval a) { return a.a > a.b ? a : Interval{ceil_div(a.a - 2, 2), floor_div(a.b + 2, 2)}; };
        need[L - 1] = band_iv(L - 1);
        for (int k = L - 2; k >= 0; --k) {
          const Interval b = band_iv(k);
          need[k + 1] = unite(need[k + 1], esup(b));
          need[k] = unite(b, rsup(need[k + 1]));
        }
        for (int k = L - 1; k >= 0; --k) {
          mneed[k] = unite(mneed[k], band_iv(k));
          if (k > 0) mneed[k - 1] = unite(mneed[k - 1], rsup(mneed[k]));
        }
        const Interval n0 = unite(need[0], mneed[0]);
        if (ax == 0) { nx0 = n0.a; nx1 = n0.b; } else { ny0 = n0.a; ny1 = n0.b; }
      }
      const Rect r0 = c.roi[0];
      Rect shrunk{};
      if (nx0 <= nx1 && ny0 <= ny1) {
        const int64_t x0 = std::max<int64_t>(r0.x, floor_div(nx0, A) * A);
        const int64_t y0 = std::max<int64_t>(r0.y, floor_div(ny0, A) * A);
        const int64_t x1 = std::min<int64_t>(r0.x + r0.w, ceil_div(nx1 + 1, A) * A);
        const int64_t y1 = std::min<int64_t>(r0.y + r0.h, ceil_div(ny1 + 1, A) * A);
        if (x0 < x1 && y0 < y1) shrunk = Rect{(int)x0, (int)y0, (int)(x1 - x0), (int)(y1 - y0)};
      }
      for (int k = 0; k < L; ++k) {
        if (shrunk.empty()) { c.roi[k] = Rect{}; c.band[k] = Rect{}; continue; }
        const int xa = shrunk.x >> k, ya = shrunk.y >> k;
        const int xb = std::min<int>(p->dw[k], (int)ceil_div(shrunk.x + shrunk.w, (int64_t)1 << k));
        const int yb = std::min<int>(p->dh[k], (int)ceil_div(shrunk.y + shrunk.h, (int64_t)1 << k));
        c.roi[k] = Rect{xa, ya, xb - xa, yb - ya};
        c.band[k] = intersect(c.band[k], c.roi[k]);
      }
    }
    // --- band storage windows: columns widened, within the roi, to whole 32-byte sectors
    //     counted from the roi's origin, where the pass's tiles start: a tile's row of the
    //     band then covers whole sectors, so no sector is written in part by two tiles ---
    const int q = 32 / p->es;
    for (int k = 0; k < L; ++k) {
      const Rect b = c.band[k], r = c.roi[k];
      if (b.empty()) { c.lwin[k] = Rect{}; continue; }
      const int x0 = r.x + (int)floor_div(b.x - r.x, q) * q;
      const int x1 = std::min<int>(r.x + r.w, r.x + (int)ceil_div(b.x + b.w - r.x, q) * q);
      c.lwin[k] = Rect{x0, b.y, x1 - x0, b.h};
    }
    // --- keep the seam weights on roi[0] ---
    const Rect r0 = c.roi[0];
    if (!r0.empty()) {
      c.mask_row = align_up(r0.w, 256);
      c.mask0.assign((size_t)c.mask_row * r0.h, 0);
      for (int y = 0; y < r0.h; ++y)
        std::memcpy(&c.mask0[(size_t)y * c.mask_row], m + (size_t)(r0.y + y) * canvas_w + r0.x, r0.w);
    }
  }
  // --- workspace layout ---
  Layout lay;
  const int es = p->es;
  for (int i = 0; i < n; ++i) {
    CamPlan& c = p->cam[i];
    if (c.roi[0].empty()) continue;
    c.off_mask0 = lay.take((size_t)c.mask_row * c.roi[0].h);
    for (int k = (L == 1 ? 0 : 1); k < L; ++k) {
      const Rect r = c.roi[k];
      c.g_row[k] = row_elems(r.w, es);
      c.g_plane[k] = c.g_row[k] * r.h;
      c.off_g[k] = lay.take((size_t)(3 * c.g_plane[k]) * es);
      if (k >= 1) {
        c.gm_row[k] = row_elems(r.w, es);
        c.off_gm[k] = lay.take((size_t)(c.gm_row[k] * r.h) * es);
      }
    }
    for (int k = 0; k + 1 < L; ++k) {
      const Rect b = c.lwin[k];
      if (b.empty()) continue;
      c.l_row[k] = row_elems(b.w, es);
      c.l_plane[k] = c.l_row[k] * b.h;
      c.off_l[k] = lay.take((size_t)(3 * c.l_plane[k]) * es);
    }
  }
  for (int k = 0; k < L; ++k) {
    if (k == 0 && !(flags & STITCH_PLAN_KEEP_R0)) continue;
    p->has_r[k] = true;
    p->r_row[k] = row_elems(p->dw[k], es);
    p->r_plane[k] = p->r_row[k] * p->dh[k];
    p->off_r[k] = lay.take((size_t)(3 * p->r_plane[k]) * es);
  }
  for (int k = 0; k + 1 < L; ++k) p->off_items[k] = lay.take((size_t)n * sizeof(PyrItem));
  for (int k = 0; k < L; ++k) p->off_bcams[k] = lay.take((size_t)n * sizeof(BlendCam));
  p->off_bitems = lay.take((size_t)L * sizeof(BlendItem));
  for (int i = 0; i < n; ++i) {
    const CamPlan& c = p->cam[i];
    for (int k = 0; k < L; ++k) {
      const bool ok = (k > 0 || fits_offsets(c.mask_row, 0, c.roi[0].h, 1)) &&
                      fits_offsets(c.g_row[k], c.g_plane[k], c.roi[k].h, 3) &&
                      fits_offsets(c.gm_row[k], 0, c.roi[k].h, 1) && fits_offsets(c.l_row[k], c.l_plane[k], c.band[k].h, 3);
      if (!ok) return fail(STITCH_E_SHAPE, "camera %d's level-%d planes span 2^31 elements or more", i, k);
    }
  }
  p->ws_bytes = lay.top;
  *out = p;
  p = nullptr;   // disarm the guard
  return STITCH_OK;
}

size_t stitch_plan_workspace_bytes(const stitch_plan* p) { return p ? p->ws_bytes : 0; }

stitch_status stitch_plan_bind(stitch_plan* p, void* workspace, size_t bytes, void* stream) {
  if (!p) return fail(STITCH_E_NULL, "plan is NULL");
  if (!workspace) return fail(STITCH_E_WORKSPACE, "workspace is NULL");
  if (((uintptr_t)workspace & 255) != 0) return fail(STITCH_E_WORKSPACE, "workspace is not 256-byte aligned");
  if (bytes < p->ws_bytes) return fail(STITCH_E_WORKSPACE, "workspace has %zu bytes, the plan needs %zu", bytes, p->ws_bytes);
  p->ws = (uint8_t*)workspace;
  build_tables(p);
  const hipStream_t s = (hipStream_t)stream;
  stitch_status st = STITCH_OK;
  for (int i = 0; i < p->n && !st; ++i) {
    const CamPlan& c = p->cam[i];
    if (!c.mask0.empty()) st = upload(p->ws + c.off_mask0, c.mask0.data(), c.mask0.size(), s, "seam weight upload");
  }
  for (int k = 0; k + 1 < p->L && !st; ++k)
    st = upload(p->ws + p->off_items[k], p->items[k].data(), p->items[k].size() * sizeof(PyrItem), s, "table upload");
  for (int k = 0; k < p->L && !st; ++k)
    st = upload(p->ws + p->off_bcams[k], p->bcams[k].data(), p->bcams[k].size() * sizeof(BlendCam), s,
                "table upload");
  if (!st)
    st = upload(p->ws + p->off_bitems, p->bitems.data(), p->bitems.size() * sizeof(BlendItem), s, "table upload");
  if (!st) {
    const hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) st = hip_fail(e, "bind synchronise");
  }
  if (st) p->ws = nullptr;
  return st;
}

stitch_status stitch_frame(stitch_plan* p, const stitch_image* frames, stitch_image* pano, void* stream) {
  if (!p) return fail(STITCH_E_NULL, "plan is NULL");
  if (!frames) return fail(STITCH_E_NULL, "frames is NULL");
  if (!p->ws) return fail(STITCH_E_STATE, "plan has no workspace bound");
  stitch_status st = check_image(pano, "pano", STITCH_U8, STITCH_HWC, 3);
  if (st) return st;
  if (pano->width != p->W || pano->height != p->H)
    return fail(STITCH_E_SHAPE, "pano is %dx%d, the plan's canvas is %dx%d", pano->width, pano->height, p->W, p->H);
  FrameArgs fa;
  if ((st = frame_args(p, frames, fa))) return st;
  const hipStream_t s = (hipStream_t)stream;
  const bool f16 = p->storage == STITCH_F16;
  const int L = p->L;
  // optional event chain: one event before the first launch and one after each launch
  auto mark = [&](int kind) { return p->timing.mark(s, kind); };
  struct EndCall {
    EventLog& log;
    ~EndCall() { log.end_call(); }
  } end_call{p->timing};
  hipError_t e;
  if ((st = mark(-1))) return st;
  if (L == 1) {
    for (int i = 0; i < p->n; ++i) {
      const CamPlan& c = p->cam[i];
      const Rect r = c.roi[0];
      if (r.empty()) continue;
      e = launch_warp(f16, fa.ptr[i], fa.row[i], c.fw, c.fh, c.hinv, r.x, r.y, p->ws + c.off_g[0], c.g_row[0],
                      c.g_plane[0], r.w, r.h, s);
      if (e != hipSuccess) return hip_fail(e, "warp launch");
      if ((st = mark(6))) return st;
    }
  }
  for (int k = 0; k + 1 < L; ++k) {
    if (p->tiles[k] <= 0) continue;
    e = launch_pyr(f16, true, k == 0, (const PyrItem*)(p->ws + p->off_items[k]), (int)p->items[k].size(),
                   p->tiles[k], fa, s, p->wg_cap[k]);
    if (e != hipSuccess) return hip_fail(e, "pyramid pass launch");
    if ((st = mark(k == 0 ? 0 : 1))) return st;
  }
  for (int k = L - 1; k >= 0; --k) {
    const BlendItem& bi = p->bitems[k];
    PanoArg po{nullptr, 0};
    if (k == 0) { po.ptr = (uint8_t*)pano->data; po.row = pano->row_pitch; }
    e = launch_blend(f16, k == 0, nullptr, 1, bi.tiles_x * bi.tiles_y, po, s, &bi);
    if (e != hipSuccess) return hip_fail(e, "blend launch");
    const int kind = k == 0 ? (L > 1 ? 2 : 5) : (k + 1 < L ? 3 : 4);
    if ((st = mark(kind))) return st;
  }
  return STITCH_OK;
}

stitch_status stitch_plan_set_timing(stitch_plan* p, int32_t enable) {
  if (!p) return fail(STITCH_E_NULL, "plan is NULL");
  p->timing.reset(enable != 0);
  return STITCH_OK;
}

stitch_status stitch_plan_read_timing(stitch_plan* p, double ms[STITCH_TIMING_KINDS],
                                      int32_t launches[STITCH_TIMING_KINDS]) {
  if (!p || !ms || !launches) return fail(STITCH_E_NULL, "plan, ms or launches is NULL");
  const stitch_status st = p->timing.collect();
  for (int i = 0; i < STITCH_TIMING_KINDS; ++i) { ms[i] = p->timing.ms[i]; launches[i] = p->timing.n[i]; }
  return st;
}

stitch_status stitch_plan_view(const stitch_plan* p, int32_t what, int32_t camera, int32_t level, stitch_image* view,
                               int32_t* origin_x, int32_t* origin_y) {
  if (!p || !view || !origin_x || !origin_y) return fail(STITCH_E_NULL, "plan, view or origin is NULL");
  if (!p->ws) return fail(STITCH_E_STATE, "plan has no workspace bound");
  if (level < 0 || level >= p->L) return fail(STITCH_E_LEVELS, "level %d outside 0..%d", level, p->L - 1);
  std::memset(view, 0, sizeof *view);
  view->layout = STITCH_CHW;
  view->dtype = p->storage;
  const int es = p->es;
  if (what == 3) {
    if (!p->has_r[level]) return fail(STITCH_E_SHAPE, "R_%d is not stored by this plan", level);
    view->data = p->ws + p->off_r[level];
    view->width = p->dw[level]; view->height = p->dh[level]; view->channels = 3;
    view->row_pitch = p->r_row[level] * es; view->plane_pitch = p->r_plane[level] * es;
    *origin_x = 0; *origin_y = 0;
    return STITCH_OK;
  }
  if (camera < 0 || camera >= p->n) return fail(STITCH_E_SHAPE, "camera %d outside 0..%d", camera, p->n - 1);
  const CamPlan& c = p->cam[camera];
  Rect r;
  if (what == 0) {
    r = c.band[level];
    *origin_x = r.x; *origin_y = r.y;
    if (r.empty()) return STITCH_OK;
    view->channels = 3;
    if (level + 1 < p->L) {
      const Rect w = c.lwin[level];   // the band inside its storage window
      view->data = p->ws + c.off_l[level] + ((int64_t)(r.y - w.y) * c.l_row[level] + (r.x - w.x)) * es;
      view->row_pitch = c.l_row[level] * es; view->plane_pitch = c.l_plane[level] * es;
    } else {
      const Rect g = c.roi[level];
      view->data = p->ws + c.off_g[level] + ((int64_t)(r.y - g.y) * c.g_row[level] + (r.x - g.x)) * es;
      view->row_pitch = c.g_row[level] * es; view->plane_pitch = c.g_plane[level] * es;
    }
  } else if (what == 1) {
    if (level == 0 && p->L > 1) return fail(STITCH_E_SHAPE, "G_0 is never stored by the fused path");
    r = c.roi[level];
    *origin_x = r.x; *origin_y = r.y;
    if (r.empty()) return STITCH_OK;
    view->channels = 3;
    view->data = p->ws + c.off_g[level];
    view->row_pitch = c.g_row[level] * es; view->plane_pitch = c.g_plane[level] * es;
  } else if (what == 2) {
    r = c.roi[level];
    *origin_x = r.x; *origin_y = r.y;
    if (r.empty()) return STITCH_OK;
    view->channels = 1;
    if (level == 0) {
      view->dtype = STITCH_U8;
      view->data = p->ws + c.off_mask0;
      view->row_pitch = c.mask_row;
    } else {
      view->data = p->ws + c.off_gm[level];
      view->row_pitch = c.gm_row[level] * es;
    }
    view->plane_pitch = view->row_pitch * r.h;
  } else {
    return fail(STITCH_E_SHAPE, "what = %d is not 0..3", what);
  }
  view->width = r.w;
  view->height = r.h;
  return STITCH_OK;
}

stitch_status stitch_plan_regions(const stitch_plan* p, int32_t camera, int32_t level, int32_t roi[4],
                                  int32_t band[4]) {
  if (!p || !roi || !band) return fail(STITCH_E_NULL, "plan, roi or band is NULL");
  if (camera < 0 || camera >= p->n) return fail(STITCH_E_SHAPE, "camera %d outside 0..%d", camera, p->n - 1);
  if (level < 0 || level >= p->L) return fail(STITCH_E_LEVELS, "level %d outside 0..%d", level, p->L - 1);
  const Rect r = p->cam[camera].roi[level], b = p->cam[camera].band[level];
  roi[0] = r.x; roi[1] = r.y; roi[2] = r.w; roi[3] = r.h;
  band[0] = b.x; band[1] = b.y; band[2] = b.w; band[3] = b.h;
  return STITCH_OK;
}

void stitch_plan_destroy(stitch_plan* p) { delete p; }

// ------------------------------------------------------------------------------------ batch

}  // extern "C"

namespace stitch {
constexpr int kMaxGroups = 8;
}

struct stitch_batch {
  int njobs = 0, maxL = 0;
  bool f16 = false;
  std::vector<stitch_plan*> plans;
  std::vector<PyrItem> pyr[kMaxLevels];
  int pyr_tiles[kMaxLevels] = {};
  size_t off_pyr[kMaxLevels] = {};
  int wg_cap[kMaxLevels] = {};                // tuned persistent workgroups per CU per phase
  int sub[kMaxLevels] = {};                   // tuned 16-row sub-steps per pyramid tile per phase
  int64_t t16[kMaxLevels] = {};               // 16-row tiles per phase (independent of sub)
  std::vector<BlendItem> blend[kMaxLevels];
  int blend_tiles[kMaxLevels] = {};
  size_t off_blend[kMaxLevels] = {};
  std::vector<int> frame_item;                // per job and camera: index into pyr[0] (or -1)
  std::vector<int> frame_job, frame_cam;
  size_t ws_bytes = 0;
  uint8_t* ws = nullptr;
  bool uploaded = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  EventLog timing;   // per-launch timing; while on, runs are launched eagerly
  // Grouped schedule (ngroups > 1): the jobs split into sub-batches; the level-0 pass of
  // group g + 1 runs on the caller's stream while group g's later passes and blends run on a
  // side stream, so the VALU-heavy warp pass of one group overlaps the memory-bound rest of
  // the previous one.  The sub-batches' tables live in this batch's workspace after its own.
  int ngroups = 1;
  std::vector<stitch_batch*> groups;
  std::vector<std::vector<int>> group_jobs;
  size_t own_bytes = 0;                       // this batch's own tables (the rest: groups)
  hipStream_t side = nullptr;
  std::vector<hipEvent_t> gev;                // per group: its level-0 pass queued; last: join
  ~stitch_batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (stitch_batch* g : groups) delete g;
    for (hipEvent_t e : gev) (void)hipEventDestroy(e);
    if (side) (void)hipStreamDestroy(side);
  }
};

namespace {

void drop_graph(stitch_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

// Enqueue the phases of the batch: pyramid passes by level (from level k_first; k_first =
// 0 starts with the warp + level-0 pass), then, with blends, the blends from the top level
// down; a job joins the phases its own level count has.
stitch_status enqueue_phases(stitch_batch* b, hipStream_t s, int k_first, int k_end, bool blends) {
  FrameArgs fa;
  std::memset(&fa, 0, sizeof fa);   // n = 0: frames come from the item tables
  stitch_status st = STITCH_OK;
  for (int k = k_first; !st && k < k_end && k + 1 < b->maxL; ++k) {
    if (b->pyr_tiles[k] <= 0) continue;
    const hipError_t e = launch_pyr(b->f16, true, k == 0, (const PyrItem*)(b->ws + b->off_pyr[k]),
                                    (int)b->pyr[k].size(), b->pyr_tiles[k], fa, s, b->wg_cap[k]);
    if (e != hipSuccess) return hip_fail(e, "batch pyramid launch");
    st = b->timing.mark(s, k);
  }
  for (int k = b->maxL - 1; blends && !st && k >= 0; --k) {
    if (b->blend_tiles[k] <= 0) continue;
    const hipError_t e = launch_blend(b->f16, k == 0, (const BlendItem*)(b->ws + b->off_blend[k]),
                                      (int)b->blend[k].size(), b->blend_tiles[k], PanoArg{nullptr, 0}, s);
    if (e != hipSuccess) return hip_fail(e, "batch blend launch");
    st = b->timing.mark(s, kMaxLevels + k);
  }
  return st;
}

// Every phase of the batch on one stream (with the per-launch timing events when enabled).
stitch_status enqueue_batch(stitch_batch* b, hipStream_t s) {
  struct EndCall {
    EventLog& log;
    ~EndCall() { log.end_call(); }
  } end_call{b->timing};
  stitch_status st = b->timing.mark(s, -1);
  if (!st) st = enqueue_phases(b, s, 0, kMaxLevels, true);
  return st;
}

// The grouped schedule: level-0 passes of the groups in turn on s; after group g's, its
// later passes and blends on the side stream; s joins the side stream at the end.
stitch_status enqueue_grouped(stitch_batch* b, hipStream_t s) {
  for (int g = 0; g < b->ngroups; ++g) {
    stitch_status st = enqueue_phases(b->groups[g], s, 0, 1, false);
    if (st) return st;
    hipError_t e = hipEventRecord(b->gev[g], s);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->side, b->gev[g], 0);
    if (e != hipSuccess) return hip_fail(e, "group fork");
    if ((st = enqueue_phases(b->groups[g], b->side, 1, kMaxLevels, true))) return st;
  }
  hipError_t e = hipEventRecord(b->gev[b->ngroups], b->side);
  if (e == hipSuccess) e = hipStreamWaitEvent(s, b->gev[b->ngroups], 0);
  return e == hipSuccess ? STITCH_OK : hip_fail(e, "group join");
}

// Check the run's frames and panoramas, write their pointers into the tables and upload
// the tables when anything changed.
stitch_status batch_prepare(stitch_batch* b, const stitch_image* const* frames, stitch_image* panos, hipStream_t s) {
  if (!b->ws) return fail(STITCH_E_STATE, "batch has no workspace bound");
  if (!frames || !panos) return fail(STITCH_E_NULL, "frames or panos is NULL");
  bool changed = !b->uploaded;
  for (int j = 0; j < b->njobs; ++j) {
    const stitch_plan* p = b->plans[j];
    if (!frames[j]) return fail(STITCH_E_NULL, "frames[%d] is NULL", j);
    char name[48];
    snprintf(name, sizeof name, "panos[%d]", j);
    stitch_status st = check_image(&panos[j], name, STITCH_U8, STITCH_HWC, 3);
    if (st) return st;
    if (panos[j].width != p->W || panos[j].height != p->H)
      return fail(STITCH_E_SHAPE, "panos[%d] does not match job %d's canvas", j, j);
    for (int i = 0; i < p->n; ++i) {
      snprintf(name, sizeof name, "frames[%d][%d]", j, i);
      st = check_image(&frames[j][i], name, STITCH_U8, STITCH_HWC, 3);
      if (st) return st;
      if (frames[j][i].width != p->cam[i].fw || frames[j][i].height != p->cam[i].fh)
        return fail(STITCH_E_SHAPE, "%s does not match the planned frame size", name);
      if (frames[j][i].row_pitch * (int64_t)frames[j][i].height >= ((int64_t)1 << 31) ||
          frames[j][i].row_pitch >= ((int64_t)1 << 24))
        return fail(STITCH_E_SHAPE, "%s spans 2 GiB or more, or its rows 16 MiB or more", name);
    }
  }
  for (size_t q = 0; q < b->frame_item.size(); ++q) {
    const stitch_image& f = frames[b->frame_job[q]][b->frame_cam[q]];
    PyrItem& it = b->pyr[0][b->frame_item[q]];
    if (it.img != f.data || it.img_row != f.row_pitch) {
      it.img = f.data;
      it.img_row = f.row_pitch;
      changed = true;
    }
  }
  for (size_t q = 0; q < b->blend[0].size(); ++q) {
    BlendItem& bi = b->blend[0][q];
    const stitch_image& pv = panos[q];
    if (bi.pano != pv.data || bi.pano_row != pv.row_pitch) {
      bi.pano = (uint8_t*)pv.data;
      bi.pano_row = pv.row_pitch;
      changed = true;
    }
  }
  if (!changed) return STITCH_OK;
  for (int k = 0; k < b->maxL; ++k) {
    stitch_status st = upload(b->ws + b->off_pyr[k], b->pyr[k].data(), b->pyr[k].size() * sizeof(PyrItem), s,
                              "batch table upload");
    if (!st) st = upload(b->ws + b->off_blend[k], b->blend[k].data(), b->blend[k].size() * sizeof(BlendItem), s,
                         "batch table upload");
    if (st) return st;
  }
  b->uploaded = true;
  return STITCH_OK;
}

// Copy the batch's per-level settings (tile height, workgroups per CU) to its groups.
void sync_groups(stitch_batch* b) {
  for (stitch_batch* g : b->groups) {
    for (int k = 0; k + 1 < g->maxL; ++k) {
      g->wg_cap[k] = b->wg_cap[k];
      if (b->sub[k] > 0 && g->sub[k] != b->sub[k]) {
        g->sub[k] = b->sub[k];
        set_sub(g->pyr[k], g->sub[k], g->pyr_tiles[k]);
        g->uploaded = false;
      }
    }
  }
}

// Point the groups' tables at their slices of the batch's workspace (after its own tables).
void bind_groups(stitch_batch* b) {
  size_t off = b->own_bytes;
  for (stitch_batch* g : b->groups) {
    g->ws = b->ws ? b->ws + off : nullptr;
    g->uploaded = false;
    off += g->ws_bytes;
  }
}

// Each group's frames and panoramas (its jobs' entries of the run's arrays) into its tables.
stitch_status prepare_groups(stitch_batch* b, const stitch_image* const* frames, stitch_image* panos, hipStream_t s) {
  std::vector<const stitch_image*> fr;
  std::vector<stitch_image> pv;
  for (int g = 0; g < b->ngroups; ++g) {
    fr.clear();
    pv.clear();
    for (int j : b->group_jobs[g]) {
      fr.push_back(frames[j]);
      pv.push_back(panos[j]);
    }
    const stitch_status st = batch_prepare(b->groups[g], fr.data(), pv.data(), s);
    if (st) return st;
  }
  return STITCH_OK;
}

uint64_t fnv1a(uint64_t h, const void* data, size_t n) {
  const uint8_t* p = (const uint8_t*)data;
  for (size_t i = 0; i < n; ++i) h = (h ^ p[i]) * 1099511628211ull;
  return h;
}

// One pyramid pass's tunable settings and where its launch table lives.
struct PassTune {
  std::vector<PyrItem>* items;   // host table (tile counts follow the sub-steps)
  uint8_t* dev_table;            // its device copy
  int* tiles;                    // the pass's tile count
  int* sub;                      // 16-row sub-steps per tile
  int* cap;                      // persistent workgroups per compute unit
  int64_t t16;                   // 16-row tiles of the pass (independent of sub)
  bool warp;                     // the level-0 pass (warp + pyramid)
};

// Use sub_k sub-steps per tile: rewrite the host table and upload it (waited for, since
// the host table is rewritten by the next choice).
stitch_status apply_sub(PassTune& pt, int sub_k, hipStream_t s) {
  *pt.sub = sub_k;
  set_sub(*pt.items, sub_k, *pt.tiles);
  stitch_status r = upload(pt.dev_table, pt.items->data(), pt.items->size() * sizeof(PyrItem), s, "table upload");
  if (r) return r;
  const hipError_t e = hipStreamSynchronize(s);
  return e == hipSuccess ? STITCH_OK : hip_fail(e, "table upload");
}

// Pick, per pass, the tile height (16 * sub rows, sub in 1, 2, 4, 8; the taller ones only
// while the pass still has a tile per compute unit) and the workgroups per compute unit
// (as many as fit, 1, 2, or one per tile) by timing every pair on the stream (the other
// passes keep their settings).  cache_path: a text file of earlier choices keyed by the
// device, the storage type, the form (salt) and every pass's 16-row tile count.
stitch_status tune_passes(int np, PassTune* passes, bool f16, const FrameArgs& fa, hipStream_t s,
                          const char* cache_path, uint64_t salt) {
  prepare_launches();
  hipDeviceProp_t prop;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return fail(STITCH_E_DEVICE, "cannot query the device");
  int64_t t16[kMaxLevels] = {};
  for (int k = 0; k < np; ++k) t16[k] = passes[k].t16;
  uint64_t key = fnv1a(1469598103934665603ull, prop.gcnArchName, strlen(prop.gcnArchName));
  key = fnv1a(key, &f16, sizeof f16);
  if (salt) key = fnv1a(key, &salt, sizeof salt);
  key = fnv1a(key, t16, sizeof t16);
  constexpr int kFields = 2 * kMaxLevels;   // per pass: sub-steps per tile, workgroups per CU
  int cached[kFields];
  bool hit = false;
  if (cache_path) {
    FILE* f = fopen(cache_path, "r");
    if (f) {
      char line[1024];
      while (!hit && fgets(line, sizeof line, f)) {
        unsigned long long k2 = 0;
        int n = 0, off = 0;
        if (sscanf(line, "%llx %d%n", &k2, &n, &off) == 2 && k2 == key && n == kFields) {
          hit = true;
          const char* q = line + off;
          for (int i = 0; i < kFields && hit; ++i) {
            int used = 0;
            if (sscanf(q, "%d%n", &cached[i], &used) != 1) hit = false;
            q += used;
          }
          for (int k = 0; k < kMaxLevels && hit; ++k)
            if (cached[2 * k] < 1 || cached[2 * k] > 8 || (cached[2 * k] & (cached[2 * k] - 1)) != 0 ||
                cached[2 * k + 1] < -1 || cached[2 * k + 1] > 2)
              hit = false;
        }
      }
      fclose(f);
    }
  }
  stitch_status st = STITCH_OK;
  if (hit) {
    for (int k = 0; k < np && !st; ++k) {
      *passes[k].cap = cached[2 * k + 1];
      st = apply_sub(passes[k], cached[2 * k], s);
    }
    return st;
  }
  const int subs[] = {1, 2, 4, 8};
  const int caps[] = {0, 1, 2, -1};
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return fail(STITCH_E_DEVICE, "event create failed");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(STITCH_E_DEVICE, "event create failed");
  }
  for (int k = 0; k < np && !st; ++k) {
    PassTune& pt = passes[k];
    if (pt.t16 <= 0) continue;
    float best = 1e30f;
    int best_sub = *pt.sub, best_cap = 0;
    for (int sub_k : subs) {
      if (sub_k > 1 && pt.t16 / sub_k < 256) continue;   // at least a tile per compute unit
      st = apply_sub(pt, sub_k, s);
      for (int c : caps) {
        float score = 1e30f;   // fastest of five launches after a warm-up one
        for (int rep = 0; rep < 6 && !st; ++rep) {
          hipError_t e = hipEventRecord(e0, s);
          if (e == hipSuccess)
            e = launch_pyr(f16, true, pt.warp, (const PyrItem*)pt.dev_table, (int)pt.items->size(), *pt.tiles, fa,
                           s, c);
          if (e == hipSuccess) e = hipEventRecord(e1, s);
          if (e == hipSuccess) e = hipEventSynchronize(e1);
          float ms = 0.0f;
          if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
          if (e != hipSuccess) st = hip_fail(e, "autotune timing");
          if (rep > 0) score = std::min(score, ms);
        }
        if (!st && score < best) {
          best = score;
          best_sub = sub_k;
          best_cap = c;
        }
      }
      if (st) break;
    }
    *pt.cap = best_cap;
    if (!st) st = apply_sub(pt, best_sub, s);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st) return st;
  if (cache_path) {
    FILE* f = fopen(cache_path, "a");
    if (f) {
      fprintf(f, "%llx %d", (unsigned long long)key, kFields);
      for (int k = 0; k < kMaxLevels; ++k)
        fprintf(f, " %d %d", k < np && *passes[k].sub > 0 ? *passes[k].sub : 1, k < np ? *passes[k].cap : 0);
      fprintf(f, "\n");
      fclose(f);
    }
  }
  return STITCH_OK;
}

// Validate caller-given settings: tile_rows[k] in {0 (keep), 16, 32, 64, 128} and
// wg_per_cu[k] in {-1, 0, 1, 2} for the np passes.
stitch_status check_config(int np, const int32_t* wg_per_cu, const int32_t* tile_rows) {
  if (!wg_per_cu || !tile_rows) return fail(STITCH_E_NULL, "wg_per_cu or tile_rows is NULL");
  for (int k = 0; k < np; ++k) {
    const int t = tile_rows[k];
    if (t != 0 && t != 16 && t != 32 && t != 64 && t != 128)
      return fail(STITCH_E_SHAPE, "tile_rows[%d] = %d is not 0, 16, 32, 64 or 128", k, t);
    if (wg_per_cu[k] < -1 || wg_per_cu[k] > 2)
      return fail(STITCH_E_SHAPE, "wg_per_cu[%d] = %d outside -1..2", k, wg_per_cu[k]);
  }
  return STITCH_OK;
}

}  // namespace

extern "C" {

stitch_status stitch_batch_create(int32_t njobs, stitch_plan* const* plans, stitch_batch** out) {
  if (!out) return fail(STITCH_E_NULL, "out is NULL");
  *out = nullptr;
  if (!plans) return fail(STITCH_E_NULL, "plans is NULL");
  if (njobs < 1) return fail(STITCH_E_SHAPE, "njobs = %d", njobs);
  stitch_batch* b = new (std::nothrow) stitch_batch();
  if (!b) return fail(STITCH_E_UNSUPPORTED, "out of host memory");
  struct Guard { stitch_batch*& b; ~Guard() { delete b; } } guard{b};
  b->njobs = njobs;
  for (int j = 0; j < njobs; ++j) {
    stitch_plan* p = plans[j];
    if (!p) return fail(STITCH_E_NULL, "plans[%d] is NULL", j);
    if (!p->ws) return fail(STITCH_E_STATE, "plans[%d] has no workspace bound", j);
    if (p->L < 2) return fail(STITCH_E_UNSUPPORTED, "plans[%d] has one level; batches need two or more", j);
    for (int q = 0; q < j; ++q)
      if (plans[q] == p) return fail(STITCH_E_SHAPE, "plans[%d] repeats plans[%d] (each job needs its own plan)", j, q);
    if (j == 0) b->f16 = p->storage == STITCH_F16;
    else if (b->f16 != (p->storage == STITCH_F16))
      return fail(STITCH_E_UNSUPPORTED, "all plans of a batch must share the storage type");
    b->plans.push_back(p);
    b->maxL = std::max(b->maxL, p->L);
  }
  for (int j = 0; j < njobs; ++j) {
    stitch_plan* p = b->plans[j];
    for (int k = 0; k + 1 < p->L; ++k)
      for (size_t q = 0; q < p->items[k].size(); ++q) {
        PyrItem it = p->items[k][q];
        it.tile_begin = b->pyr_tiles[k];
        b->pyr_tiles[k] += it.tiles_x * it.tiles_y;
        if (k == 0) {
          b->frame_item.push_back((int)b->pyr[0].size());
          b->frame_job.push_back(j);
          b->frame_cam.push_back(it.frame_slot);
          it.img = nullptr;
          it.img_row = 0;
        }
        b->pyr[k].push_back(it);
      }
  }
  // one sub-step choice per pass, from the batch's own 16-row tile count
  for (int k = 0; k + 1 < b->maxL; ++k) {
    for (const PyrItem& it : b->pyr[k]) b->t16[k] += (int64_t)it.tiles_x * it.rows16;
    b->sub[k] = choose_sub(b->t16[k]);
    set_sub(b->pyr[k], b->sub[k], b->pyr_tiles[k]);
  }
  // blends: level-0 items in job order, so blend[0][j] belongs to job j
  for (int k = 0; k < b->maxL; ++k)
    for (int j = 0; j < njobs; ++j) {
      stitch_plan* p = b->plans[j];
      if (k >= p->L) continue;
      BlendItem bi = p->bitems[k];
      bi.tile_begin = b->blend_tiles[k];
      b->blend_tiles[k] += bi.tiles_x * bi.tiles_y;
      b->blend[k].push_back(bi);
    }
  Layout lay;
  for (int k = 0; k < b->maxL; ++k) {
    b->off_pyr[k] = lay.take(std::max<size_t>(1, b->pyr[k].size()) * sizeof(PyrItem));
    b->off_blend[k] = lay.take(std::max<size_t>(1, b->blend[k].size()) * sizeof(BlendItem));
  }
  b->own_bytes = lay.top;
  // room for the tables of up to kMaxGroups groups (stitch_batch_set_groups): together they
  // hold every item once, plus each group's per-level alignment
  b->ws_bytes = 2 * b->own_bytes + (size_t)kMaxGroups * 2 * kMaxLevels * 256;
  *out = b;
  b = nullptr;
  return STITCH_OK;
}

size_t stitch_batch_workspace_bytes(const stitch_batch* b) { return b ? b->ws_bytes : 0; }

stitch_status stitch_batch_bind(stitch_batch* b, void* workspace, size_t bytes) {
  if (!b) return fail(STITCH_E_NULL, "batch is NULL");
  if (!workspace) return fail(STITCH_E_WORKSPACE, "workspace is NULL");
  if (((uintptr_t)workspace & 255) != 0) return fail(STITCH_E_WORKSPACE, "workspace is not 256-byte aligned");
  if (bytes < b->ws_bytes) return fail(STITCH_E_WORKSPACE, "workspace has %zu bytes, the batch needs %zu", bytes, b->ws_bytes);
  b->ws = (uint8_t*)workspace;
  b->uploaded = false;
  bind_groups(b);
  drop_graph(b);
  return STITCH_OK;
}

stitch_status stitch_batch_run(stitch_batch* b, const stitch_image* const* frames, stitch_image* panos, void* stream) {
  if (!b) return fail(STITCH_E_NULL, "batch is NULL");
  const hipStream_t s = (hipStream_t)stream;
  stitch_status st = batch_prepare(b, frames, panos, s);
  if (st) return st;
  // the null stream cannot be captured, and timing events stay out of graphs: launch eagerly
  if (!s || b->timing.on) return enqueue_batch(b, s);
  const bool grouped = b->ngroups > 1;
  if (grouped && (st = prepare_groups(b, frames, panos, s))) return st;
  if (!b->exec) {
    prepare_launches();
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "batch capture begin");
    st = grouped ? enqueue_grouped(b, s) : enqueue_batch(b, s);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(s, &g);
    if (st) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return hip_fail(e, "batch capture end");
    b->graph = g;
    e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      drop_graph(b);
      return hip_fail(e, "batch graph instantiate");
    }
  }
  const hipError_t e = hipGraphLaunch(b->exec, s);
  return e == hipSuccess ? STITCH_OK : hip_fail(e, "batch graph launch");
}

stitch_status stitch_batch_autotune(stitch_batch* b, const stitch_image* const* frames, stitch_image* panos,
                                    void* stream, const char* cache_path) {
  if (!b) return fail(STITCH_E_NULL, "batch is NULL");
  const hipStream_t s = (hipStream_t)stream;
  stitch_status st = batch_prepare(b, frames, panos, s);
  if (st) return st;
  drop_graph(b);
  PassTune passes[kMaxLevels];
  int np = 0;
  for (int k = 0; k + 1 < b->maxL; ++k)
    passes[np++] = PassTune{&b->pyr[k], b->ws + b->off_pyr[k], &b->pyr_tiles[k], &b->sub[k], &b->wg_cap[k],
                            b->t16[k], k == 0};
  FrameArgs fa;
  std::memset(&fa, 0, sizeof fa);   // n = 0: frames come from the item tables
  st = tune_passes(np, passes, b->f16, fa, s, cache_path, 0x62617463ull /* batch */);
  sync_groups(b);
  return st;
}

stitch_status stitch_batch_config(const stitch_batch* b, int32_t wg_per_cu[STITCH_MAX_LEVELS],
                                  int32_t tile_rows[STITCH_MAX_LEVELS]) {
  if (!b || !wg_per_cu || !tile_rows) return fail(STITCH_E_NULL, "batch, wg_per_cu or tile_rows is NULL");
  for (int k = 0; k < kMaxLevels; ++k) {
    wg_per_cu[k] = b->wg_cap[k];
    tile_rows[k] = k + 1 < b->maxL ? kPyrTY * b->sub[k] : 0;
  }
  return STITCH_OK;
}

stitch_status stitch_batch_set_timing(stitch_batch* b, int32_t enable) {
  if (!b) return fail(STITCH_E_NULL, "batch is NULL");
  b->timing.reset(enable != 0);
  return STITCH_OK;
}

stitch_status stitch_batch_read_timing(stitch_batch* b, double ms[STITCH_BATCH_TIMING_KINDS],
                                       int32_t launches[STITCH_BATCH_TIMING_KINDS]) {
  if (!b || !ms || !launches) return fail(STITCH_E_NULL, "batch, ms or launches is NULL");
  const stitch_status st = b->timing.collect();
  for (int i = 0; i < STITCH_BATCH_TIMING_KINDS; ++i) { ms[i] = b->timing.ms[i]; launches[i] = b->timing.n[i]; }
  return st;
}

void stitch_batch_destroy(stitch_batch* b) { delete b; }

stitch_status stitch_batch_set_config(stitch_batch* b, const int32_t wg_per_cu[STITCH_MAX_LEVELS],
                                      const int32_t tile_rows[STITCH_MAX_LEVELS]) {
  if (!b) return fail(STITCH_E_NULL, "batch is NULL");
  const int np = std::max(0, b->maxL - 1);
  stitch_status st = check_config(np, wg_per_cu, tile_rows);
  if (st) return st;
  for (int k = 0; k < np; ++k) {
    b->wg_cap[k] = wg_per_cu[k];
    if (tile_rows[k]) {
      b->sub[k] = tile_rows[k] / kPyrTY;
      set_sub(b->pyr[k], b->sub[k], b->pyr_tiles[k]);
    }
  }
  b->uploaded = false;   // the next run uploads the tables and captures a new graph
  sync_groups(b);
  drop_graph(b);
  return STITCH_OK;
}

stitch_status stitch_batch_set_groups(stitch_batch* b, int32_t ngroups) {
  if (!b) return fail(STITCH_E_NULL, "batch is NULL");
  if (ngroups < 1 || ngroups > kMaxGroups || ngroups > b->njobs)
    return fail(STITCH_E_SHAPE, "groups = %d outside 1..%d (and at most the %d jobs)", ngroups, kMaxGroups, b->njobs);
  drop_graph(b);
  for (stitch_batch* g : b->groups) delete g;
  b->groups.clear();
  b->group_jobs.clear();
  b->ngroups = 1;
  if (ngroups == 1) return STITCH_OK;
  // longest-processing-time split by level-0 work (16-row tiles of the warp pass), each
  // group's jobs in their batch order
  std::vector<int64_t> work(b->njobs, 0);
  for (size_t q = 0; q < b->pyr[0].size(); ++q)
    work[b->frame_job[q]] += (int64_t)b->pyr[0][q].tiles_x * b->pyr[0][q].rows16;
  std::vector<int> order(b->njobs);
  for (int j = 0; j < b->njobs; ++j) order[j] = j;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return work[x] > work[y]; });
  std::vector<int64_t> load(ngroups, 0);
  b->group_jobs.assign(ngroups, {});
  for (int j : order) {
    const int g = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    b->group_jobs[g].push_back(j);
    load[g] += std::max<int64_t>(work[j], 1);
  }
  for (auto& v : b->group_jobs) std::sort(v.begin(), v.end());
  size_t need = b->own_bytes;
  for (int g = 0; g < ngroups; ++g) {
    std::vector<stitch_plan*> pl;
    for (int j : b->group_jobs[g]) pl.push_back(b->plans[j]);
    stitch_batch* sub = nullptr;
    stitch_status st = stitch_batch_create((int32_t)pl.size(), pl.data(), &sub);
    if (st) {
      for (stitch_batch* x : b->groups) delete x;
      b->groups.clear();
      b->group_jobs.clear();
      return st;
    }
    b->groups.push_back(sub);
    need += sub->own_bytes;
    sub->ws_bytes = sub->own_bytes;   // a group holds only its own tables
  }
  if (need > b->ws_bytes) {   // cannot happen: create reserved room for kMaxGroups groups
    for (stitch_batch* x : b->groups) delete x;
    b->groups.clear();
    b->group_jobs.clear();
    return fail(STITCH_E_WORKSPACE, "group tables need %zu bytes, the batch reserved %zu", need, b->ws_bytes);
  }
  if (!b->side) {
    const hipError_t e = hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "side stream");
  }
  while ((int)b->gev.size() < kMaxGroups + 1) {
    hipEvent_t ev;
    const hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "group events");
    b->gev.push_back(ev);
  }
  b->ngroups = ngroups;
  bind_groups(b);
  sync_groups(b);
  return STITCH_OK;
}

int32_t stitch_batch_group_count(const stitch_batch* b) { return b ? b->ngroups : 0; }

// ------------------------------------------------------------------------------------ plan settings

// Upload the pyramid-pass tables of a bound plan and wait for them.
static stitch_status plan_upload_items(stitch_plan* p, hipStream_t s) {
  for (int k = 0; k + 1 < p->L; ++k) {
    const stitch_status st =
        upload(p->ws + p->off_items[k], p->items[k].data(), p->items[k].size() * sizeof(PyrItem), s, "table upload");
    if (st) return st;
  }
  const hipError_t e = hipStreamSynchronize(s);
  return e == hipSuccess ? STITCH_OK : hip_fail(e, "table upload");
}

stitch_status stitch_plan_config(const stitch_plan* p, int32_t wg_per_cu[STITCH_MAX_LEVELS],
                                 int32_t tile_rows[STITCH_MAX_LEVELS]) {
  if (!p || !wg_per_cu || !tile_rows) return fail(STITCH_E_NULL, "plan, wg_per_cu or tile_rows is NULL");
  for (int k = 0; k < kMaxLevels; ++k) {
    const bool pass = k + 1 < p->L;
    wg_per_cu[k] = pass ? p->wg_cap[k] : 0;
    tile_rows[k] = pass ? kPyrTY * (p->sub[k] > 0 ? p->sub[k] : (p->sub_req[k] > 0 ? p->sub_req[k] : 1)) : 0;
  }
  return STITCH_OK;
}

stitch_status stitch_plan_set_config(stitch_plan* p, const int32_t wg_per_cu[STITCH_MAX_LEVELS],
                                     const int32_t tile_rows[STITCH_MAX_LEVELS], void* stream) {
  if (!p) return fail(STITCH_E_NULL, "plan is NULL");
  const int np = std::max(0, p->L - 1);
  stitch_status st = check_config(np, wg_per_cu, tile_rows);
  if (st) return st;
  for (int k = 0; k < np; ++k) {
    p->wg_cap[k] = wg_per_cu[k];
    if (tile_rows[k]) {
      p->sub_req[k] = tile_rows[k] / kPyrTY;
      if (p->ws) {
        p->sub[k] = p->sub_req[k];
        set_sub(p->items[k], p->sub[k], p->tiles[k]);
      }
    }
  }
  return p->ws ? plan_upload_items(p, (hipStream_t)stream) : STITCH_OK;
}

stitch_status stitch_autotune(stitch_plan* p, const stitch_image* frames, void* stream, const char* cache_path) {
  if (!p) return fail(STITCH_E_NULL, "plan is NULL");
  if (!frames) return fail(STITCH_E_NULL, "frames is NULL");
  if (!p->ws) return fail(STITCH_E_STATE, "plan has no workspace bound");
  FrameArgs fa;
  stitch_status st = frame_args(p, frames, fa);
  if (st) return st;
  PassTune passes[kMaxLevels];
  int np = 0;
  for (int k = 0; k + 1 < p->L; ++k) {
    int64_t t16 = 0;
    for (const PyrItem& it : p->items[k]) t16 += (int64_t)it.tiles_x * it.rows16;
    passes[np++] = PassTune{&p->items[k], p->ws + p->off_items[k], &p->tiles[k], &p->sub[k], &p->wg_cap[k], t16,
                            k == 0};
  }
  st = tune_passes(np, passes, p->storage == STITCH_F16, fa, (hipStream_t)stream, cache_path,
                   0x706c61696eull /* plain */);
  for (int k = 0; k < np; ++k) p->sub_req[k] = p->sub[k];   // kept across rebinds
  return st;
}

}  // extern "C"
