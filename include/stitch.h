/*
 * stitch.h -- C ABI of the per-frame panorama stitching path on MI355X (gfx950).
 *
 * The path is the one the paper runs once registration has fixed each camera's
 * transformation: every camera frame is transformed onto the panorama with its
 * pre-corrected parameters (Alg. 4, step 1), and the transformed frames are blended
 * into the panorama (Alg. 4, step 6) with multi-band fusion to remove seams
 * (Sec. 1, contribution 3).  Buffers are sized once when the system starts and
 * reused for every frame (Sec. 4.3.2, space pre-allocation); work is queued
 * asynchronously on a caller stream (Sec. 4.3.2, operation queues).
 *
 * Definitions used by every call (the paper gives none of them; these are the
 * readings of the textbook Burt-Adelson multiresolution spline):
 *   - pixel (x, y) = (column, row) is a sample at integer coordinates;
 *   - a homography H (row-major 3x3, double) maps source pixels to canvas pixels;
 *     the warp pulls each canvas pixel through adj(H)/adj(H)[2][2] rounded to FP32,
 *     with FP32 coordinate arithmetic (no fused multiply-add, IEEE divide); a
 *     sample with non-positive homogeneous z is 0;
 *   - bilinear interpolation of u8/255; taps outside the source contribute 0;
 *   - REDUCE: 5x5 separable [1,4,6,4,1]/16 filter, keep even samples, sides
 *     ceil(n/2); EXPAND: zero-insert at even fine samples, same filter times 4;
 *     borders reflect-101 (-i -> i, n-1+i -> n-1-i), folded in the fine domain;
 *     every level side must be >= 3;
 *   - Laplacian level L_k = G_k - EXPAND(G_{k+1}), top level L_{L-1} = G_{L-1};
 *   - blend: B_k = sum_i Gm_i^k * L_i^k over cameras, R_{L-1} = B_{L-1},
 *     R_k = B_k + EXPAND(R_{k+1}), panorama = clamp(rint(255 R_0), 0, 255).
 *
 * Memory.  Every data pointer is DEVICE memory owned by the caller (frames,
 * panorama, pyramids, workspace); the library owns only the host-side plan and
 * batch objects.  All work is enqueued on the given stream (a hipStream_t; NULL is
 * the null stream) with no implicit device synchronisation, except where a call
 * says otherwise.
 *
 * Errors.  Every call returns a stitch_status.  Argument errors are detected on the
 * host before anything is enqueued; a HIP launch failure returns STITCH_E_DEVICE.
 * Faults during asynchronous execution surface at the caller's next
 * synchronisation.  stitch_last_error() returns a thread-local message describing
 * the last failure on the calling thread.  No C++ exception crosses this ABI.
 * Distinct plans may be used from distinct threads; one plan is not re-entrant.
 */
#ifndef STITCH_H
#define STITCH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define STITCH_ABI_VERSION 1
#define STITCH_MAX_LEVELS 16
#define STITCH_MAX_CAMERAS 64

typedef enum {
  STITCH_OK = 0,
  STITCH_E_NULL = 1,        /* a required pointer is NULL */
  STITCH_E_SHAPE = 2,       /* sizes, channels, layout, pitch or dtype inconsistent */
  STITCH_E_LEVELS = 3,      /* level count outside 1..16 or a level side < 3 */
  STITCH_E_HOMOGRAPHY = 4,  /* non-finite H, or adj(H)[2][2] == 0 */
  STITCH_E_MASK = 5,        /* seam weights do not sum to 255 at some canvas pixel */
  STITCH_E_WORKSPACE = 6,   /* workspace NULL, too small or not 256-byte aligned */
  STITCH_E_DEVICE = 7,      /* a HIP runtime call failed */
  STITCH_E_UNSUPPORTED = 8, /* a dtype/layout combination or a case the library does not provide */
  STITCH_E_STATE = 9        /* object used in the wrong state (e.g. plan not bound) */
} stitch_status;

typedef enum { STITCH_U8 = 0, STITCH_F16 = 1, STITCH_F32 = 2 } stitch_dtype;
typedef enum { STITCH_HWC = 0, STITCH_CHW = 1 } stitch_layout;

/* A caller-owned device image.  HWC: pixel (x, y) channel c at
 * data + y*row_pitch + (x*channels + c)*elem.  CHW: at
 * data + c*plane_pitch + y*row_pitch + x*elem.  Pitches are in BYTES. */
typedef struct {
  void*   data;
  int32_t width, height, channels;
  int32_t dtype;          /* stitch_dtype */
  int32_t layout;         /* stitch_layout */
  int64_t row_pitch;
  int64_t plane_pitch;    /* CHW only */
} stitch_image;

/* A pyramid whose level k covers a rectangle of the level-k canvas.  The level-k
 * canvas has sides ceil(canvas/2^k).  level[k] element (0,0) sits at level-k canvas
 * coordinates (origin_x[k], origin_y[k]); samples of the full-canvas array outside
 * the stored rectangle are taken as 0. */
typedef struct {
  int32_t levels;
  int32_t canvas_w, canvas_h;
  int32_t origin_x[STITCH_MAX_LEVELS];
  int32_t origin_y[STITCH_MAX_LEVELS];
  stitch_image level[STITCH_MAX_LEVELS];
} stitch_levels;

typedef struct stitch_plan stitch_plan;

/* ---- library ---------------------------------------------------------------- */
int32_t     stitch_abi_version(void);                 /* STITCH_ABI_VERSION */
const char* stitch_status_str(stitch_status status);  /* static string */
const char* stitch_last_error(void);                  /* thread-local, never NULL */

/* ---- single stages ------------------------------------------------------------ */

/* Alg. 4, step 1: transform one camera frame onto the canvas.
 * src: U8 HWC, 3 channels, the camera frame.  H: source -> canvas.
 * dst: F32 or F16 CHW, 3 channels; receives G_0 on canvas pixels
 * [roi_x, roi_x + dst->width) x [roi_y, roi_y + dst->height).  Any roi is allowed
 * (the warp is pointwise).  Errors: NULL, SHAPE, HOMOGRAPHY, UNSUPPORTED, DEVICE. */
stitch_status stitch_warp(const stitch_image* src, const double H[9], int32_t roi_x, int32_t roi_y,
                          stitch_image* dst, void* stream);

/* Diagnostic of the warp's coordinate step: writes the FP32 source coordinates
 * x (plane 0) and y (plane 1) that stitch_warp computes for canvas pixels of the
 * rectangle [roi_x, roi_x+width) x [roi_y, roi_y+height) into xy (F32 CHW, 2 channels);
 * pixels with non-positive z get NaN.  Errors as stitch_warp. */
stitch_status stitch_warp_coords(const double H[9], int32_t roi_x, int32_t roi_y, stitch_image* xy,
                                 void* stream);

/* Multi-band fusion, analysis side: the Gaussian (kind 0) or Laplacian (kind 1)
 * pyramid of one image.  g0: level 0, either F32/F16 CHW with 1..3 channels or a U8
 * single-channel weight map (read as u8/255).  out: levels, canvas size, origins and
 * level images preallocated by the caller; out->level[k] has the dtype of out->level[0]
 * (F32 or F16, CHW, channels of g0), covers the rectangle given by its origin and size,
 * and receives G_k (kind 0) or L_k (kind 1).  g0 covers the rectangle of level 0.  The
 * result equals the full-canvas definition when g0 is zero outside its rectangle and
 * each level's rectangle holds that level's support; with origin 0 and full-canvas
 * sizes it is the plain pyramid of g0.  Level 0 of the output is overwritten with
 * G_0 (kind 0) or L_0 (kind 1) and may alias g0 when dtypes match.  Each output level's
 * planes must span fewer than 2^31 elements and its rows fewer than 2^23 (SHAPE
 * otherwise: the kernels address levels with 32-bit offsets).
 * workspace: device memory of stitch_pyramid_workspace_bytes(levels) bytes, 256-byte
 * aligned, holding the launch tables (calls that may overlap must not share it; the
 * table upload comes from pageable host memory and may wait for the stream).
 * Errors: NULL, SHAPE, LEVELS, WORKSPACE, UNSUPPORTED, DEVICE. */
size_t        stitch_pyramid_workspace_bytes(int32_t levels);
stitch_status stitch_pyramid(const stitch_image* g0, int32_t kind, stitch_levels* out, void* workspace,
                             size_t workspace_bytes, void* stream);

/* Multi-band fusion, synthesis side (Alg. 4, step 6): blend n (1..64) Laplacian pyramids
 * with n Gaussian weight pyramids and collapse to the panorama.
 * bands[i]: F32/F16 CHW 3-channel Laplacian levels; weights[i]: Gaussian weight
 * levels (F32/F16 1 channel of the band dtype, or U8 at any level read as u8/255); all
 * pyramids share levels and canvas size, and each level's samples outside its stored
 * rectangle count as 0; every band level's planes, and every weight level, must span
 * fewer than 2^31 elements with rows under 2^23 elements (SHAPE otherwise: 32-bit offsets).
 * pano: U8 HWC 3 channels, canvas_w x canvas_h.  keep_r: a
 * full-canvas pyramid (origins 0, band dtype, CHW, 3 channels) receiving R_k; it is
 * required when levels > 1 (the collapse reads R_{k+1} from it); its level[0].data may be
 * NULL to skip storing R_0.  workspace: stitch_blend_workspace_bytes(n, levels) bytes of
 * 256-byte aligned device memory for the launch tables (same sharing rule as
 * stitch_pyramid).  Errors: NULL, SHAPE, LEVELS, WORKSPACE, UNSUPPORTED, DEVICE. */
size_t        stitch_blend_workspace_bytes(int32_t n, int32_t levels);
stitch_status stitch_blend(int32_t n, const stitch_levels* bands, const stitch_levels* weights,
                           stitch_image* pano, stitch_levels* keep_r, void* workspace,
                           size_t workspace_bytes, void* stream);

/* ---- the whole frame, planned once (Sec. 4.3.2: pre-allocation at start-up) --- */

#define STITCH_PLAN_KEEP_R0 1   /* flags bit: also store R_0 (float) in the workspace */

/* Validate a fixed rig and plan the per-frame work: n cameras of frame_w[i] x frame_h[i]
 * (width >= 3),
 * H (n*9 doubles, source -> canvas, row-major per camera), seam weights masks[i]
 * (host, canvas_h x canvas_w uint8, row-major, summing to 255 at every pixel),
 * levels L (1..16, every canvas level side >= 3), storage STITCH_F32 or STITCH_F16 for
 * every stored pyramid level.  Host-only: touches no GPU.  The plan keeps what it
 * needs from masks; the caller may free them after the call.  Every camera's stored
 * level planes must span fewer than 2^31 elements with rows under 2^23 (SHAPE otherwise).
 * Errors: NULL, SHAPE, LEVELS, HOMOGRAPHY, MASK, UNSUPPORTED. */
stitch_status stitch_plan_create(int32_t n, const int32_t* frame_w, const int32_t* frame_h,
                                 const double* H, const uint8_t* const* masks, int32_t canvas_w,
                                 int32_t canvas_h, int32_t levels, int32_t storage, int32_t flags,
                                 stitch_plan** out);

/* Bytes of device workspace the plan needs (256-byte aligned base required). */
size_t stitch_plan_workspace_bytes(const stitch_plan* plan);

/* Attach a caller-owned device workspace and upload the plan's tables and seam
 * weights into it on the stream; returns after the stream has drained (the only call
 * that synchronises).  The workspace stays attached until rebind or destroy.
 * Errors: NULL, WORKSPACE, DEVICE. */
stitch_status stitch_plan_bind(stitch_plan* plan, void* workspace, size_t bytes, void* stream);

/* Stitch one frame set: frames[i] U8 HWC 3-channel of the planned size (each under
 * 2 GiB with rows under 16 MiB), pano U8 HWC 3-channel canvas_w x canvas_h.  Enqueues
 * warp + pyramids + mask pyramids + blend + collapse.  Errors: NULL, SHAPE, STATE (not
 * bound), DEVICE. */
stitch_status stitch_frame(stitch_plan* plan, const stitch_image* frames, stitch_image* pano,
                           void* stream);

/* Views into the bound workspace (for inspection and tests).  what: 0 = L_k of camera
 * i (3 ch), 1 = G_k of camera i (3 ch, k >= 1), 2 = Gm_k of camera i (1 ch; k = 0 is the
 * U8 weight crop), 3 = R_k (3 ch, k >= 1, or k = 0 with STITCH_PLAN_KEEP_R0).  Fills
 * view (device pointer into the workspace) and the level-k canvas origin of its element
 * (0,0).  An empty region returns width or height 0.  Errors: NULL, SHAPE, STATE. */
stitch_status stitch_plan_view(const stitch_plan* plan, int32_t what, int32_t camera, int32_t level,
                               stitch_image* view, int32_t* origin_x, int32_t* origin_y);

/* Level-k rectangle the plan computes camera i's pyramid on (roi) and the rectangle
 * where its seam weights are non-zero (band window), in level-k canvas coordinates
 * as {x, y, w, h}.  Host-only.  Errors: NULL, SHAPE. */
stitch_status stitch_plan_regions(const stitch_plan* plan, int32_t camera, int32_t level,
                                  int32_t roi[4], int32_t band[4]);

/* Per-launch timing of stitch_frame (tracing; the paper only analyses grid sizes and
 * memory, Sec. 4.3.2).  While enabled, stitch_frame records one HIP event on its stream
 * before its first launch and one after every launch, and the time between consecutive
 * events is charged to the launch's kind:
 *   0 warp + level-0 pyramid pass, 1 pyramid passes of levels >= 1, 2 blend of level 0
 *   (with EXPAND of R_1), 3 blend of a middle level, 4 blend of the top level, 5 blend of
 *   a single-level plan, 6 warp of a single-level plan.
 * set_timing clears the totals; read_timing waits for the recorded events and returns
 * accumulated milliseconds and launch counts per kind.  Errors: NULL, DEVICE. */
#define STITCH_TIMING_KINDS 8
stitch_status stitch_plan_set_timing(stitch_plan* plan, int32_t enable);
stitch_status stitch_plan_read_timing(stitch_plan* plan, double ms[STITCH_TIMING_KINDS],
                                      int32_t launches[STITCH_TIMING_KINDS]);

/* Settings of the plan's pyramid passes (the plain form, stitch_frame), as for batches:
 * pass k from level k (k = 0: warp + level 0) runs tiles of tile_rows[k] rows (16, 32, 64
 * or 128) on wg_per_cu[k] persistent workgroups per compute unit (-1: one per tile, 0: as
 * many as fit, 1, 2).  Until set or tuned, the planner picks the tallest tile that leaves
 * about eight tiles per compute unit and as many workgroups as fit.  The results do not
 * depend on the settings.  stitch_plan_config reads them (0 for levels with no pass).
 * stitch_plan_set_config sets them (tile_rows[k] = 0 keeps pass k's height); on a bound plan
 * it uploads the changed tables on the stream and waits for them.  Errors: NULL, SHAPE,
 * DEVICE. */
stitch_status stitch_plan_config(const stitch_plan* plan, int32_t wg_per_cu[STITCH_MAX_LEVELS],
                                 int32_t tile_rows[STITCH_MAX_LEVELS]);
stitch_status stitch_plan_set_config(stitch_plan* plan, const int32_t wg_per_cu[STITCH_MAX_LEVELS],
                                     const int32_t tile_rows[STITCH_MAX_LEVELS], void* stream);
/* Autotuner of the plain form (the paper sizes its thread grids by analysing the resources
 * an image needs, Sec. 4.3.2; here they are measured): times every (tile height, workgroups
 * per compute unit) pair of each pyramid pass of stitch_frame on these frames (U8 HWC, as for
 * stitch_frame) and keeps the fastest; synchronises the stream.  cache_path (optional): a
 * text file of earlier choices keyed by the device, the storage type and the plan's tile
 * counts; a hit skips the timing, a miss appends the new choice.  The choice survives a
 * rebind.  Errors: NULL, SHAPE, STATE (not bound), DEVICE. */
stitch_status stitch_autotune(stitch_plan* plan, const stitch_image* frames, void* stream, const char* cache_path);

void stitch_plan_destroy(stitch_plan* plan);

/* ---- many jobs in one captured launch sequence --------------------------------- */

/* A batch stitches several planned jobs (rigs of any camera count, resolution and level
 * count >= 2) per run.  The paper overlaps images of different resolutions with CUDA
 * stream queues (Sec. 4.3.2); here all jobs' work of one pyramid level (or one blend
 * level) is one launch over a table of per-job tiles, the launches of a run are captured
 * once into a HIP graph, and later runs replay it.  Frame and panorama pointers live in
 * the device tables (re-uploaded only when they change), so replays never need a new
 * capture.  The batch uses each plan's bound workspace for the jobs' pyramids: while a
 * plan belongs to a batch, do not run stitch_frame on it concurrently with the batch. */
typedef struct stitch_batch stitch_batch;

/* plans: njobs distinct, bound plans of one storage type.  Host-only.
 * Errors: NULL, SHAPE, STATE (a plan not bound), UNSUPPORTED (a one-level plan, mixed
 * storage types). */
stitch_status stitch_batch_create(int32_t njobs, stitch_plan* const* plans, stitch_batch** out);
size_t        stitch_batch_workspace_bytes(const stitch_batch* batch);   /* launch tables */
/* Attach caller-owned device memory (256-byte aligned) for the tables.  Host-only;
 * discards a captured graph.  Errors: NULL, WORKSPACE. */
stitch_status stitch_batch_bind(stitch_batch* batch, void* workspace, size_t bytes);
/* One run: frames[j] is job j's array of its plan's camera frames (U8 HWC), panos[j] its
 * panorama.  On a non-null stream the first run captures a graph and every run launches
 * it; on the null stream the launches are issued directly.  Errors: NULL, SHAPE, STATE,
 * DEVICE. */
stitch_status stitch_batch_run(stitch_batch* batch, const stitch_image* const* frames, stitch_image* panos,
                               void* stream);
/* Pick, for every pyramid level of the batch, the tile height of its pass (16, 32, 64 or
 * 128 rows, the taller ones only while the level still has a tile per compute unit) and
 * how many persistent workgroups per compute unit it launches (as many as fit, 1, 2, or
 * one per tile) by timing the pairs on these inputs (synchronises the stream).  cache_path (optional): a text file of
 * earlier choices keyed by device and batch geometry; a hit skips the timing and a miss
 * appends the new choice.  Errors: NULL, SHAPE, STATE, DEVICE. */
stitch_status stitch_batch_autotune(stitch_batch* batch, const stitch_image* const* frames, stitch_image* panos,
                                    void* stream, const char* cache_path);
/* Per-launch timing of stitch_batch_run (tracing, as for plans).  While enabled, runs are
 * launched eagerly (no graph) with one HIP event before the first launch and one after
 * every launch; kind k < 16 is the pyramid pass from level k (k = 0: warp + level 0), kind
 * 16 + k the blend of level k.  set_timing clears the totals; read_timing waits for the
 * recorded events and returns accumulated milliseconds and launch counts per kind.
 * Errors: NULL, DEVICE. */
#define STITCH_BATCH_TIMING_KINDS (2 * STITCH_MAX_LEVELS)
stitch_status stitch_batch_set_timing(stitch_batch* batch, int32_t enable);
stitch_status stitch_batch_read_timing(stitch_batch* batch, double ms[STITCH_BATCH_TIMING_KINDS],
                                       int32_t launches[STITCH_BATCH_TIMING_KINDS]);
/* The per-level settings in use: workgroups per CU (0: as many as fit, -1: one per tile)
 * and the pass's tile height in rows (0 for levels with no pass from them).  Errors: NULL. */
stitch_status stitch_batch_config(const stitch_batch* batch, int32_t wg_per_cu[STITCH_MAX_LEVELS],
                                  int32_t tile_rows[STITCH_MAX_LEVELS]);
/* Set the per-level settings directly instead of timing them: for every pass k (levels
 * 0 .. max levels - 2) tile_rows[k] in {16, 32, 64, 128} (0 keeps the current height) and
 * wg_per_cu[k] in {-1 (one workgroup per tile), 0 (as many as fit), 1, 2}.  The results do
 * not depend on the settings.  Host-only; the next run uploads the tables and captures a
 * new graph.  Errors: NULL, SHAPE. */
stitch_status stitch_batch_set_config(stitch_batch* batch, const int32_t wg_per_cu[STITCH_MAX_LEVELS],
                                      const int32_t tile_rows[STITCH_MAX_LEVELS]);
/* Run the jobs as `groups` (1..8, at most the job count) sub-batches balanced by their
 * warp-pass work, software-pipelined over the caller's stream and a side stream the batch
 * owns (default priority): the warp + level-0 pass of group g + 1 is queued on the caller's
 * stream while group g's later pyramid passes and blends run on the side stream, so the
 * arithmetic-heavy warp pass of one group can overlap the memory-bound passes of another (the
 * paper overlaps images of different sizes on stream queues, Sec. 4.3.2).  1 restores the
 * single sequence.  Runs on a non-null stream only (captured into one graph with the fork
 * and join); timed runs and the null stream use the single sequence.  The results do not
 * depend on the grouping.  Needs a bound batch; discards a captured graph.
 * stitch_batch_group_count returns the current count (0 for NULL).
 * Errors: NULL, SHAPE, STATE, WORKSPACE, DEVICE. */
stitch_status stitch_batch_set_groups(stitch_batch* batch, int32_t groups);
int32_t       stitch_batch_group_count(const stitch_batch* batch);
void          stitch_batch_destroy(stitch_batch* batch);

/* ---- stream-pipelined frame sequences: host frames in, host panoramas out -------- */

/* The paper keeps the upload of the next frames, the stitching of the current ones and
 * the download of the previous panorama in flight together on stream queues (Sec. 4.3.2,
 * Fig. 3).  A pipe uses `depth` (1..8) device slots, each holding one frame set and one
 * panorama of a bound plan, in a caller-owned device workspace of
 * stitch_pipe_workspace_bytes(plan, depth) bytes (256-byte aligned; the paper's start-up
 * pre-allocation, Sec. 4.3.2; 0 on bad arguments), and owns three streams of default
 * priority: copies in, stitch_frame, copies out.  Events order the reuse of a slot: its
 * frames are overwritten only after the stitch that read them, its panorama only after the
 * copy that read it.  The plan and the workspace must stay alive, and the plan bound and
 * unused by other calls, while a pipe runs on it.
 * Errors: NULL, SHAPE (depth), WORKSPACE (NULL, misaligned or too small), STATE (plan
 * without workspace), DEVICE. */
typedef struct stitch_pipe stitch_pipe;
size_t        stitch_pipe_workspace_bytes(const stitch_plan* plan, int32_t depth);
stitch_status stitch_pipe_create(stitch_plan* plan, int32_t depth, void* workspace, size_t bytes,
                                 stitch_pipe** out);
/* Stitch nframes frame sets: frames[t * n + i] is camera i's frame of set t (host memory,
 * U8 HWC with packed rows: frame_w x frame_h x 3 bytes), panos[t] its panorama (host, U8
 * HWC packed, canvas_w x canvas_h x 3 bytes).  Returns when every panorama is on the host.
 * Memory from stitch_host_alloc (pinned) lets the copies overlap the stitching; pageable
 * memory gives the same results with serialised copies.  Errors: NULL, SHAPE (nframes < 0),
 * DEVICE, and those of stitch_frame. */
stitch_status stitch_pipe_run(stitch_pipe* pipe, int32_t nframes, const uint8_t* const* frames,
                              uint8_t* const* panos);
void          stitch_pipe_destroy(stitch_pipe* pipe);
/* Pinned host memory for pipe inputs and outputs (hipHostMalloc); release it with
 * stitch_host_free.  Errors: NULL, DEVICE. */
stitch_status stitch_host_alloc(size_t bytes, void** out);
void          stitch_host_free(void* p);

/* ---- differentiable form: refining a pair's transformation -------------------- */

/* The paper fixes each frame's transformation by feature matching and PROSAC (Alg. 3,
 * Alg. 4 step 5) and stitches with it (Alg. 4 step 6).  This form makes the stitched
 * result differentiable so that the transformation of a pair can be refined by gradient
 * descent on it.  For two FLOAT frames (F32 CHW, 3 channels, values in [0, 1]) it
 * evaluates, in FP64 with the forward path's FP32 source coordinates,
 *   loss = 1/(6|Omega|) sum_{p in Omega, c} (P_c - A_c)^2 + (P_c - B_c)^2
 * where A, B are the warped frames G_0 (Alg. 4 step 6, bilinear with zero taps outside),
 * P is R_0 of their multi-band blend (Alg. 4 step 1 and step 6, before quantisation) and
 * Omega is the set of canvas pixels where both frames have all four bilinear taps inside
 * and z > 0.  Bilinear cells (floor of the source coordinates) and Omega are frozen by
 * stitch_grad_freeze, so the loss is smooth in the maps; backward returns the exact
 * gradient of that frozen loss.  Canvases up to 2^26 pixels; intended for pairs, not
 * for the throughput path. */
typedef struct stitch_grad stitch_grad;

/* frame_w/frame_h: the two frames' sizes.  masks: two HOST arrays of canvas_h x
 * canvas_w U8 seam weights summing to 255 per pixel (copied).  levels >= 1, every level's
 * sides >= 3.  Host-only.  Errors: NULL, LEVELS, SHAPE, MASK. */
stitch_status stitch_grad_create(const int32_t frame_w[2], const int32_t frame_h[2], const uint8_t* const* masks,
                                 int32_t canvas_w, int32_t canvas_h, int32_t levels, stitch_grad** out);
size_t        stitch_grad_workspace_bytes(const stitch_grad* grad);
/* Attach caller-owned device memory (256-byte aligned, >= workspace_bytes) and build the
 * seam-weight pyramids in it; synchronises the stream.  Errors: NULL, WORKSPACE, DEVICE. */
stitch_status stitch_grad_bind(stitch_grad* grad, void* workspace, size_t bytes, void* stream);
/* Freeze the bilinear cells and Omega at the source -> canvas homographies H (2 x 9,
 * row-major); writes |Omega| to omega_count (optional).  Synchronises the stream.
 * Errors: NULL, STATE (not bound), HOMOGRAPHY, SHAPE (|Omega| = 0), DEVICE. */
stitch_status stitch_grad_freeze(stitch_grad* grad, const double H[18], int64_t* omega_count, void* stream);
/* Loss at the homographies H with the frozen cells.  The frame pointers are kept for
 * stitch_grad_backward: the frames must stay alive and unchanged until it has run.
 * Synchronises the stream.  Errors: NULL, STATE (not frozen), SHAPE, UNSUPPORTED,
 * HOMOGRAPHY, DEVICE. */
stitch_status stitch_grad_forward(stitch_grad* grad, const stitch_image* frames, const double H[18], double* loss,
                                  void* stream);
/* Gradient of the last forward's loss: d_frames[i] (F32 CHW, 3 channels, the frame's
 * size; overwritten) receives d loss / d frame i, d_map (host) receives d loss / d M_i
 * (row-major, 9 per camera), M_i being the FP32 canvas -> source map adj(H_i)/adj(H_i)[2][2]
 * the warp uses.  The frame transpose gathers over the canvas pixels whose frozen cell holds
 * each source pixel, so the result is repeatable bit for bit; UNSUPPORTED when a map the
 * cells were frozen at magnifies a source pixel over about 20 times or reaches its horizon
 * over the frame.  Synchronises the stream.  Errors: NULL, STATE, SHAPE, UNSUPPORTED,
 * DEVICE. */
stitch_status stitch_grad_backward(stitch_grad* grad, stitch_image* d_frames, double d_map[18], void* stream);
/* The last forward's gradients as the upstream terms of stitch_frame_backward: d_pano =
 * dl/dP and d_warped[i] = dl/dG_0 of frame i taken directly (the loss's own terms on the
 * warped frames), each F32 CHW, 3 channels, canvas-sized; queued on the stream.  Feeding
 * them to stitch_frame_backward with a plan of the pair at the frozen maps gives this loss's
 * gradient.  Errors: NULL, STATE, SHAPE, DEVICE. */
stitch_status stitch_grad_upstream(stitch_grad* grad, stitch_image* d_pano, stitch_image* d_warped, void* stream);
void          stitch_grad_destroy(stitch_grad* grad);

/* The whole path of a plan as a differentiable function of FLOAT frames: for frames F_i
 * (F32 CHW, 3 channels, the planned sizes, values in [0, 1]) the blended and collapsed
 * panorama before quantisation, R_0 = F(F_1..F_n, M_1..M_n) (Alg. 4 steps 1 and 6, with the
 * definitions at the top of this file), where M_i is the FP32 canvas -> source map the warp
 * uses.  Every array lives on the whole canvas in FP64; the bilinear cell of a canvas pixel
 * is floor of its FP32 source coordinates at the plan's maps (the right derivative at
 * integers) and the fraction x - floor(x) is the FP32 one, as in stitch_frame.  Meant for
 * refining registration (Alg. 3 / Alg. 4 step 5 give the maps), not for the throughput path:
 * canvases up to 2^26 pixels.  The plan needs no bound workspace; both calls take a
 * workspace of stitch_frame_backward_workspace_bytes(plan) bytes (256-byte aligned; about
 * 140 bytes per canvas pixel; 0 on bad arguments).
 *
 * stitch_frame_forward_f32: r0 (F32 CHW, 3 channels, canvas size) receives R_0.  Queued on
 * the stream (waits only for the upload of each camera's seam weights).
 * Errors: NULL, SHAPE, WORKSPACE, HOMOGRAPHY, DEVICE. */
size_t        stitch_frame_backward_workspace_bytes(const stitch_plan* plan);
stitch_status stitch_frame_forward_f32(stitch_plan* plan, const stitch_image* frames, stitch_image* r0,
                                       void* workspace, size_t workspace_bytes, void* stream);
/* Vector-Jacobian product of F: given d_pano = dl/dR_0 (F32 CHW, 3 channels, canvas size)
 * and optionally d_warped (NULL, or n images of which those with data NULL are skipped:
 * dl/dG_0 of camera i taken directly on its warped frame, F32 CHW canvas-sized), writes
 * d_frames[i] = dl/dF_i (F32 CHW, the frame's size; overwritten) and d_hinv[9 i + j] =
 * dl/dM_i[j] (HOST, n x 9 doubles, row-major).  The frame transpose gathers over the canvas
 * pixels whose cell holds each source pixel (deterministic, no atomics); maps that magnify a
 * source pixel more than about 20 times, or whose horizon crosses a frame, return
 * UNSUPPORTED.  Synchronises the stream.  Errors: NULL, SHAPE, WORKSPACE, HOMOGRAPHY,
 * UNSUPPORTED, DEVICE. */
stitch_status stitch_frame_backward(stitch_plan* plan, const stitch_image* frames, const stitch_image* d_pano,
                                    const stitch_image* d_warped, stitch_image* d_frames, double* d_hinv,
                                    void* workspace, size_t workspace_bytes, void* stream);

/* Corner parameterisation of a homography (host, FP64): H (h33 = 1) is the direct linear
 * transform taking the frame corners (0,0), (w-1,0), (w-1,h-1), (0,h-1) to the canvas
 * points q = (X0,Y0, X1,Y1, X2,Y2, X3,Y3).  Errors: NULL, SHAPE, HOMOGRAPHY (degenerate). */
stitch_status stitch_corners_to_h(const double q[8], int32_t w, int32_t h, double H[9]);
/* Chain rule from d loss / d M (M = H(q)^-1 normalised to M22 = 1, as above) to
 * d loss / d q.  Errors: NULL, HOMOGRAPHY. */
stitch_status stitch_map_grad_to_corners(const double q[8], int32_t w, int32_t h, const double d_map[9],
                                         double d_q[8]);

/* ---- L-ORB features in the detection areas (registration front end) ------------ */

/* The feature detection areas of n frames from the cameras' rough alignment (Alg. 2, step
 * 1; Sec. 4.1: the areas are where the pre-aligned neighbouring frames overlap).  Host-only:
 * touches no GPU.  Camera i's footprint is the bounding box of its frame rectangle's
 * corners (0,0), (w,0), (w,h), (0,h) mapped by H_i (row-major, source -> canvas, as for
 * stitch_plan_create).  For every pair i < j whose footprints overlap with positive area,
 * the overlap, widened by `margin` canvas pixels on every side and clipped to the canvas
 * [0, canvas_w] x [0, canvas_h], is mapped back into each frame of the pair through
 * adj(H_k); the bounding box of its corner images, rounded outward with a slack of 1e-6
 * sample and clipped to the frame, is one area (x, y, width, height) of frame k when it
 * is not empty.  Each frame's areas follow the partner camera's index.  The footprint (or
 * an overlap's corner images) is bounded only when the projective depth has one sign,
 * never zero, at its four corners: a camera with an unbounded footprint gets no areas,
 * and an overlap whose corner images in frame k are unbounded gives frame k its whole
 * rectangle.  All arithmetic is FP64.
 * frame_w, frame_h: n sides (1 .. 2^20); n in 1..64; canvas sides 1 .. 2^20; margin 0 .. 2^20.
 * Outputs (HOST): counts[n] the areas of each frame (0 .. max_areas), areas[n][max_areas][4]
 *   with frame k's areas at areas + 4 k max_areas (entries past counts[k] not written);
 *   max_areas >= 1 (n - 1 is always enough).  The result feeds stitch_lorb and
 *   stitch_lorb_multi directly.
 * Errors: NULL, SHAPE (also more areas in a frame than max_areas), HOMOGRAPHY (a
 *   non-finite entry of H). */
stitch_status stitch_detection_areas(int32_t n, const int32_t* frame_w, const int32_t* frame_h, const double* H,
                                     int32_t canvas_w, int32_t canvas_h, int32_t margin, int32_t max_areas,
                                     int32_t* counts, int32_t* areas);


/* L-ORB (Sec. 4.1, Alg. 1 and Alg. 2): in each of m feature detection areas of a frame
 * (Alg. 2, step 1: the pre-aligned overlap of neighbouring cameras), FAST corners scored
 * by the Harris response, non-maximal suppression, the n_max strongest, and a BRIEF
 * descriptor for each.  The paper leaves the operators and constants open; this call
 * fixes them so that every decision is exact integer arithmetic:
 *   - gray level g = (77 R + 150 G + 29 B + 128) >> 8;
 *   - FAST: at least 9 cyclically contiguous pixels of the radius-3, 16-pixel circle all
 *     brighter than g + fast_threshold or all darker than g - fast_threshold;
 *   - gradients Ix = g(x+1,y) - g(x-1,y), Iy = g(x,y+1) - g(x,y-1); the Gaussian weighting
 *     (sigma = 1) is the 5x5 binomial window b b^T, b = [1,4,6,4,1], unnormalised, giving
 *     A, B, C; the response (alpha = 3/64, scaled by 64) R = 64 (A B - C^2) - 3 (A + B)^2;
 *   - candidates: FAST corners with R >= harris_threshold (Alg. 1 step 5 deletes those below it); a candidate survives when every
 *     candidate among its 8 neighbours has a smaller R, or an equal R and a later raster
 *     position; the n_max survivors of largest R are kept, equal R in raster order;
 *   - BRIEF (Sec. 4.1.2) on S = b b^T * g: pair k of the pattern (dx1, dy1, dx2, dy2, each
 *     clamped to -15..15) gives bit k of the "greater" string when S(p + d1) > S(p + d2)
 *     and of the "less" string when S(p + d1) < S(p + d2) (the paper's three-valued test).
 * Only points 17 or more samples from every frame edge are considered (the descriptor
 * support); areas are clipped to that range, and an area clipped to nothing yields none.
 *
 * frame: U8 HWC, 3 channels, device, spanning under 2 GiB; sides >= 35.
 * areas: HOST array of m (1..64) rectangles (x, y, width, height) in frame coordinates,
 *   width, height >= 0; each clipped area holds under 2^30 samples.
 * pattern: DEVICE array of nd x 4 int32 offsets; nd a multiple of 32 in 32..512.
 * Outputs (DEVICE, area i at offset i times the per-area size): counts[m] the number kept
 *   (<= n_max, 1..2^20), points[m][n_max][2] their (x, y) in frame coordinates,
 *   responses[m][n_max] their R, descriptors[m][n_max][2 nd/32] words of the "greater"
 *   string then of the "less" string, bit k in bit k%32 of word k/32.  Entries past
 *   counts[i] are not written.
 * workspace: device, 256-byte aligned, at least stitch_lorb_workspace_bytes for the same
 *   frame size and areas (24 bytes per area sample; a host-only query, 0 on bad
 *   arguments).
 * Work is queued on `stream` as five kernel launches covering all areas (no allocation,
 * no memory set, no synchronisation).  Selection histograms the survivors' responses and
 * ranks only the survivors in the histogram buckets that hold the n_max strongest, by
 * comparing every pair of them: its cost grows with the square of that set (n_max plus
 * one bucket's share).
 * Errors: NULL, SHAPE (also a pattern not 16-byte aligned), WORKSPACE, DEVICE. */
size_t        stitch_lorb_workspace_bytes(int32_t frame_w, int32_t frame_h, int32_t m, const int32_t* areas);
stitch_status stitch_lorb(const stitch_image* frame, int32_t m, const int32_t* areas, int32_t fast_threshold,
                          int64_t harris_threshold, int32_t n_max, int32_t nd, const int32_t* pattern,
                          int32_t* counts, int32_t* points, int64_t* responses, uint32_t* descriptors,
                          void* workspace, size_t workspace_bytes, void* stream);

/* The same for the areas of several frames at once (e.g. every camera of a frame set):
 * one call, five launches covering all of them.  frames: HOST array of nframes (1..16)
 * frame descriptions (device data, each as for stitch_lorb); m_per_frame: HOST, the number
 * of areas of each frame (>= 0, 1..64 in total); areas: HOST, all frames' rectangles in
 * frame order, each in its own frame's coordinates.  Outputs and workspace as for
 * stitch_lorb, indexed by the area's position in `areas`; the results equal one stitch_lorb
 * per frame.  Errors as stitch_lorb. */
size_t        stitch_lorb_multi_workspace_bytes(int32_t nframes, const int32_t* frame_w, const int32_t* frame_h,
                                                const int32_t* m_per_frame, const int32_t* areas);
stitch_status stitch_lorb_multi(int32_t nframes, const stitch_image* frames, const int32_t* m_per_frame,
                                const int32_t* areas, int32_t fast_threshold, int64_t harris_threshold,
                                int32_t n_max, int32_t nd, const int32_t* pattern, int32_t* counts, int32_t* points,
                                int64_t* responses, uint32_t* descriptors, void* workspace, size_t workspace_bytes,
                                void* stream);

/* Per-launch timing of stitch_lorb and stitch_lorb_multi (diagnostics), process-wide.  While enabled, each call
 * records a HIP event on its stream before its first launch and after each of its five
 * launches: 0 clear the counts, 1 detection (FAST, response, suppression), 2 selection
 * threshold, 3 ranking, 4 BRIEF.  set_timing clears the totals; read_timing waits for the
 * recorded events and returns accumulated milliseconds and launch counts per launch.
 * Errors: NULL, DEVICE. */
#define STITCH_LORB_KINDS 5
stitch_status stitch_lorb_set_timing(int32_t enable);
stitch_status stitch_lorb_read_timing(double ms[STITCH_LORB_KINDS], int32_t launches[STITCH_LORB_KINDS]);

/* ---- pairwise registration: multi-probe LSH matching and PROSAC ----------------- */

/* Multi-probe LSH matching (Sec. 4.2.1; Alg. 3, step 1) of the L-ORB descriptors of area A
 * (queries) against those of area B (references), e.g. the facing overlap areas of two
 * neighbouring cameras.  Readings fixed here (the paper names the method only):
 *   - distance: L1 of the ternary descriptors = popcount(gt ^ gt') + popcount(lt ^ lt');
 *   - LSH: bit sampling of the "greater" string; table l's key has bit b equal to gt bit
 *     positions[l * kbits + b];
 *   - probes: in every table the query's own key and the kbits keys one bit away; the
 *     candidates are the union over tables;
 *   - a query's match is its nearest candidate by (distance, reference index), kept when
 *     the distance is at most max_dist.
 * desc_a / desc_b: DEVICE rows of 2 nd/32 uint32 (stitch_lorb's layout), 8-byte aligned;
 * count_a / count_b: DEVICE int32, the valid rows (stitch_lorb's counts[i]), capped at
 * cap_a / cap_b (1..65536).  tables 1..16, kbits 0..24 (0: every point is a candidate,
 * i.e. exhaustive search); positions: HOST tables x kbits int32 in 0..nd-1.
 * match / dist: DEVICE int32[cap_a]: reference index and distance, -1 where there is no
 * match and for rows past count_a.  workspace: stitch_lsh_match_workspace_bytes (the keys),
 * 256-byte aligned.  Errors: NULL, SHAPE, WORKSPACE, DEVICE. */
size_t        stitch_lsh_match_workspace_bytes(int32_t cap_a, int32_t cap_b, int32_t tables);
stitch_status stitch_lsh_match(int32_t nd, const uint32_t* desc_a, const int32_t* count_a, int32_t cap_a,
                               const uint32_t* desc_b, const int32_t* count_b, int32_t cap_b, int32_t tables,
                               int32_t kbits, const int32_t* positions, int32_t max_dist, int32_t* match,
                               int32_t* dist, void* workspace, size_t workspace_bytes, void* stream);

/* PROSAC screening of the matches and the transformation they yield (Sec. 4.2.2; Alg. 3,
 * step 2; Alg. 4, step 5).  Readings fixed here:
 *   - quality order: matches by (distance, query index); samples of 4;
 *   - the growth function of Chum and Matas with T_N, evaluated in FP64 in the order
 *     T_4 = T_N prod_{i<4} (4-i)/(M-i), T_{n+1} = T_n (n+1)/(n+1-4), T'_4 = 1,
 *     T'_{n+1} = T'_n + ceil(T_{n+1} - T_n); hypothesis t (1-based) grows n when t = T'_n
 *     and n < M, then samples the n-th match and 3 draws from the top n-1 unless T'_n < t
 *     (then 4 draws from the top n);
 *   - draws from the caller's uniforms: draw k of a range of R takes
 *     r = min(floor(u_k (R - k)), R - k - 1) and the r-th index not drawn before (values
 *     outside [0, 1) are clamped into the range);
 *   - model: 4-point DLT with h33 = 1 (FP64); a sample with three collinear points in
 *     either frame is skipped; inliers: w > 0 and squared reprojection error <= eps^2;
 *   - a fixed budget of nhyp hypotheses; the best has the most inliers (ties: the earlier);
 *     H is the least-squares DLT over its inliers on Hartley-normalised coordinates (5 or
 *     more inliers), else the best's own model; no valid hypothesis: H = 0, 0 inliers.
 * pts_a: DEVICE int32 [cap_a][2], pts_b: DEVICE int32 [cap_b][2] (stitch_lorb's points);
 * match, dist, count_a: as stitch_lsh_match wrote them (any distances below INT32_MAX).  uniforms: DEVICE double
 * [nhyp][4] in [0, 1) (the random draws are an input); nhyp 1..65536.  eps > 0 and
 * 0 < T_N <= 2^53 (the schedule is integer-valued; SHAPE otherwise).
 * Outputs (DEVICE): H[9] double row-major (frame A -> frame B, h33 = 1), inliers (int32),
 * inlier_mask uint8[cap_a] (1 where query i's match is an inlier of the best hypothesis),
 * hyp_counts int32[nhyp] (each hypothesis' inlier count, 0 when skipped).
 * workspace: stitch_prosac_workspace_bytes, 256-byte aligned.
 * Errors: NULL, SHAPE, WORKSPACE, DEVICE. */
size_t        stitch_prosac_workspace_bytes(int32_t cap_a, int32_t nhyp);
/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): stitch_prosac without a workspace
 * argument.  Its scratch is a 1 MiB array the library holds on each device it runs on until
 * the process ends; calls whose stitch_prosac_workspace_bytes(cap_a, nhyp) exceeds 1 MiB
 * (cap_a 4096 with more than 12,280 hypotheses, for instance) return SHAPE.  Every call on
 * a device shares that device's array: calls that overlap on one GPU (other streams, other
 * threads) race, so serialise them.  The kernels write every scratch value before reading it.  It allocates
 * nothing (the array's address is looked up on the first call on each device).  Outputs and
 * errors as stitch_prosac. */
stitch_status stitch_prosac_noalloc(const int32_t* pts_a, const int32_t* pts_b, int32_t cap_b, const int32_t* match,
                                    const int32_t* dist, const int32_t* count_a, int32_t cap_a, int32_t nhyp,
                                    const double* uniforms, double T_N, double eps, double* H, int32_t* inliers,
                                    uint8_t* inlier_mask, int32_t* hyp_counts, void* stream);
stitch_status stitch_prosac(const int32_t* pts_a, const int32_t* pts_b, int32_t cap_b, const int32_t* match,
                            const int32_t* dist, const int32_t* count_a, int32_t cap_a, int32_t nhyp,
                            const double* uniforms, double T_N, double eps, double* H, int32_t* inliers,
                            uint8_t* inlier_mask, int32_t* hyp_counts, void* workspace, size_t workspace_bytes,
                            void* stream);

/* ---- every camera pair of a rig in one launch per stage ----------------------------- */

/* Matching and PROSAC of several area pairs at once (Alg. 3 for every neighbouring pair of
 * a rig; the paper overlaps its images on stream queues, Sec. 4.3.2): one launch per stage
 * covers all pairs, each pair computed exactly as by stitch_lsh_match / stitch_prosac with
 * the same settings (results equal bit for bit).  The pair tables are HOST arrays of npairs
 * (1..256) entries; every pointer inside them is DEVICE memory with the meaning, layout and
 * limits of the single-pair call.  Up to 16 pairs travel to the kernels as launch arguments
 * (the call then allocates, copies and waits for nothing and can be captured into a graph);
 * more are uploaded into the head of the workspace on the stream first (not for graph
 * capture).  Then two (matching) or three (PROSAC) kernels are launched.
 * workspace: stitch_lsh_match_multi_workspace_bytes / stitch_prosac_multi_workspace_bytes
 *   (0 on bad arguments), 256-byte aligned, caller-owned.
 * Errors: NULL, SHAPE, WORKSPACE, DEVICE (as the single-pair calls, per pair). */
typedef struct {
  const uint32_t* desc_a;  /* cap_a rows of descriptors (stitch_lorb's layout) */
  const int32_t* count_a;  /* rows in use */
  int32_t cap_a;
  const uint32_t* desc_b;
  const int32_t* count_b;
  int32_t cap_b;
  int32_t* match;          /* [cap_a] outputs */
  int32_t* dist;           /* [cap_a] */
} stitch_match_pair;
size_t        stitch_lsh_match_multi_workspace_bytes(int32_t npairs, const stitch_match_pair* pairs, int32_t tables);
stitch_status stitch_lsh_match_multi(int32_t npairs, const stitch_match_pair* pairs, int32_t nd, int32_t tables,
                                     int32_t kbits, const int32_t* positions, int32_t max_dist, void* workspace,
                                     size_t workspace_bytes, void* stream);

typedef struct {
  const int32_t* pts_a;     /* [cap_a][2] */
  const int32_t* pts_b;     /* [cap_b][2] */
  int32_t cap_b;
  const int32_t* match;     /* [cap_a], as stitch_lsh_match wrote it */
  const int32_t* dist;      /* [cap_a] */
  const int32_t* count_a;
  int32_t cap_a;
  const double* uniforms;   /* [nhyp][4] */
  double* H;                /* [9] outputs */
  int32_t* inliers;         /* [1] */
  uint8_t* inlier_mask;     /* [cap_a] */
  int32_t* hyp_counts;      /* [nhyp] */
} stitch_prosac_pair;
size_t        stitch_prosac_multi_workspace_bytes(int32_t npairs, const stitch_prosac_pair* pairs, int32_t nhyp);
stitch_status stitch_prosac_multi(int32_t npairs, const stitch_prosac_pair* pairs, int32_t nhyp, double T_N,
                                  double eps, void* workspace, size_t workspace_bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* STITCH_H */
