// Internal descriptors shared by the host runtime (stitch_api.cpp) and the gfx950
// kernels (kernels.hip).  Plain structs: they are copied to device memory or passed
// as kernel arguments.
#pragma once
#include <stdint.h>
#include <hip/hip_runtime.h>

#include "stitch.h"

namespace stitch {

constexpr int kMaxLevels = 16;
constexpr int kMaxCameras = 64;

// Tile shape of the fused pyramid pass and of the blend pass (level-k pixels).
constexpr int kPyrTX = 64, kPyrTY = 16;
constexpr int kBlendTX = 64, kBlendTY = 16;
constexpr int kThreads = 256;

enum SrcKind : int32_t { kSrcNone = 0, kSrcWarp = 1, kSrcPlanes = 2, kSrcU8 = 3 };

struct Hinv9 { float h[9]; };

// One camera's tile range in a fused REDUCE (+ EXPAND/subtract) pass from level k
// to level k+1.  Level-k input covers roi (zero outside it, reflect-101 at canvas
// edges) except for a warp source, which is evaluated wherever it is needed.
struct PyrItem {
  int32_t tile_begin, tiles_x, tiles_y;
  int32_t tile_x0, tile_y0;               // level-k origin of tile (0,0); both even
  int32_t fine_w, fine_h;                 // level-k canvas sides
  int32_t roi_x, roi_y, roi_w, roi_h;     // level-k input rectangle
  // image source (channels nch)
  int32_t img_kind, nch;
  const void* img;                        // planes (storage type) or u8 HWC frame
  int64_t img_row, img_plane;             // elements (planes) / bytes (frame row)
  int32_t frame_w, frame_h, frame_slot, pad0;
  float hinv[9];
  // weight (mask) source, one channel
  int32_t msk_kind, pad1;
  const void* msk;                        // u8 plane or storage-type plane on roi
  int64_t msk_row;                        // elements
  // outputs at level k+1 on croi
  int32_t croi_x, croi_y, croi_w, croi_h;
  void* g_out;  int64_t g_row, g_plane;   // nch planes
  void* gm_out; int64_t gm_row;           // 1 plane
  // Laplacian band at level k on the window lw (w == 0: not written)
  int32_t lw_x, lw_y, lw_w, lw_h;
  void* l_out;  int64_t l_row, l_plane;
  // a tile is kPyrTX columns by sub * kPyrTY rows; rows16 = 16-row blocks of the item
  int32_t sub, rows16;
};

// Per-call frame pointers of the fused level-0 pass (kernel argument).
struct FrameArgs {
  int32_t n, pad;
  const uint8_t* ptr[kMaxCameras];
  int64_t row[kMaxCameras];               // bytes
};

// One camera's contribution to a blend level.
struct BlendCam {
  const void* lap; int64_t lap_row, lap_plane;   // storage type, 3 planes
  int32_t lx, ly, lw, lh;                         // band rectangle (level-k canvas)
  const void* wgt; int64_t wgt_row;               // weights: storage type or u8
  int32_t wgt_u8, pad;
  int32_t wx, wy, ww, wh;                         // weight rectangle
};

// One canvas level of one stitch job in a blend launch; a launch covers the tiles of
// several items (jobs), tile_begin being each item's first tile.
struct BlendItem {
  int32_t tile_begin, tiles_x, tiles_y;
  int32_t W, H;                     // level-k canvas sides
  int32_t cW, cH;                   // level-(k+1) canvas sides (used when has_coarse)
  int32_t ncam, has_coarse, pad;
  const BlendCam* cams;             // device array of ncam cameras
  const void* r_in; int64_t rin_row, rin_plane;    // R_{k+1} (storage type)
  void* r_out; int64_t rout_row, rout_plane;       // R_k (storage type) or nullptr
  uint8_t* pano; int64_t pano_row;                 // U8 HWC (level 0) or nullptr
};

// Launchers (kernels.hip).  f16 selects half-precision storage.
// warp: level-0 pass whose image source is the homography warp (always emits L_0).
// wg_per_cu: persistent workgroups per compute unit (0: as many as fit, < 0: one per tile).
hipError_t launch_pyr(bool f16, bool emit_lap, bool warp, const PyrItem* items_dev, int nitems, int total_tiles,
                      const FrameArgs& frames, hipStream_t s, int wg_per_cu = 0);
// Runs the occupancy queries the launchers cache, so later launches (e.g. inside a stream
// capture) make no device queries.
void prepare_launches();
// Table sizes the kernels accept.
constexpr int kMaxBlendCams = kMaxCameras;
// Per-call panorama of a single-item level-0 launch (kernel argument; ptr == nullptr:
// every item's own pano field is used).
struct PanoArg {
  uint8_t* ptr;
  int64_t row;
};

// final_level: level 0, which writes the uint8 panorama of every item.
// one != nullptr: a single item passed by value (items_dev unused).
hipError_t launch_blend(bool f16, bool final_level, const BlendItem* items_dev, int nitems, int total_tiles,
                        const PanoArg& po, hipStream_t s, const BlendItem* one = nullptr);
hipError_t launch_warp(bool f16, const uint8_t* src, int64_t src_row, int w, int h, const float* hinv9,
                       int roi_x, int roi_y, void* dst, int64_t dst_row, int64_t dst_plane, int dw, int dh,
                       hipStream_t s);
hipError_t launch_warp_coords(const float* hinv9, int roi_x, int roi_y, float* dst, int64_t row,
                              int64_t plane, int dw, int dh, hipStream_t s);
hipError_t launch_expand_sub(bool f16, int nch, void* fine, int64_t f_row, int64_t f_plane, int fx, int fy,
                             int fw, int fh, const void* coarse, int64_t c_row, int64_t c_plane, int cx,
                             int cy, int cw, int ch, int canvas_w, int canvas_h, hipStream_t s);
hipError_t launch_convert(bool f16_out, int nch, bool src_u8, const void* src, int64_t s_row, int64_t s_plane,
                          void* dst, int64_t d_row, int64_t d_plane, int w, int h, hipStream_t s);

// Geometry of a plan for the other host files: cameras, their frame sizes (arrays of at
// least kMaxCameras), the canvas, and whether a workspace is bound.
void plan_geometry(const stitch_plan* p, int* n, int* frame_w, int* frame_h, int* canvas_w, int* canvas_h,
                   bool* bound);

// One camera of a plan for the float-frame forward and its vector-Jacobian product: frame
// size, the FP32 canvas -> source map and the seam weights on their support box (weights
// holds ww x wh bytes row-major, or is NULL when the camera has no weight anywhere).
struct PlanCamera {
  int fw, fh;
  float hinv[9];
  int wx, wy, ww, wh;
  const uint8_t* weights;
};
int plan_levels(const stitch_plan* p);
void plan_camera(const stitch_plan* p, int i, PlanCamera* out);

// Host helpers shared by the API files (stitch_api.cpp).
stitch_status fail(stitch_status s, const char* fmt, ...);
stitch_status hip_fail(hipError_t e, const char* what);
stitch_status check_image(const stitch_image* im, const char* name, int dtype, int layout, int channels);
bool hinv_spec(const double* H, float out[9], double* sign_out, const char** why);

}  // namespace stitch
