// Stream-pipelined frame sequences (host frames in, host panoramas out): the upload of a
// frame set, its stitching and the download of its panorama run on three streams, so the
// copies of neighbouring frame sets overlap the stitching of the current one (the stream
// queues of Sec. 4.3.2, Fig. 3).
#include <hip/hip_runtime.h>

#include <cstring>
#include <new>
#include <vector>

#include "stitch_internal.h"

using namespace stitch;

struct stitch_pipe {
  stitch_plan* plan = nullptr;
  int depth = 0, n = 0, W = 0, H = 0;
  int fw[kMaxCameras] = {}, fh[kMaxCameras] = {};
  hipStream_t s_in = nullptr, s_comp = nullptr, s_out = nullptr;
  std::vector<void*> frames;   // depth x n device frames, packed rows (in the caller's workspace)
  std::vector<void*> panos;    // depth device panoramas, packed rows (in the caller's workspace)
  std::vector<hipEvent_t> ev_in, ev_comp, ev_out;   // per slot: copied in, stitched, copied out
};

namespace {

void release(stitch_pipe* q) {
  for (hipStream_t s : {q->s_in, q->s_comp, q->s_out})
    if (s) (void)hipStreamSynchronize(s);
  for (auto* v : {&q->ev_in, &q->ev_comp, &q->ev_out})
    for (hipEvent_t e : *v)
      if (e) (void)hipEventDestroy(e);
  for (hipStream_t s : {q->s_in, q->s_comp, q->s_out})
    if (s) (void)hipStreamDestroy(s);
  delete q;
}

size_t round256(size_t v) { return (v + 255) / 256 * 256; }

// Bytes of one slot (a frame set and a panorama, each buffer 256-byte aligned).
size_t slot_bytes(int n, const int* fw, const int* fh, int W, int H) {
  size_t b = 0;
  for (int i = 0; i < n; ++i) b += round256((size_t)fw[i] * fh[i] * 3);
  return b + round256((size_t)W * H * 3);
}

}  // namespace

extern "C" {

size_t stitch_pipe_workspace_bytes(const stitch_plan* plan, int32_t depth) {
  if (!plan || depth < 1 || depth > 8) return 0;
  int n = 0, W = 0, H = 0, fw[kMaxCameras], fh[kMaxCameras];
  bool bound = false;
  plan_geometry(plan, &n, fw, fh, &W, &H, &bound);
  return (size_t)depth * slot_bytes(n, fw, fh, W, H);
}

stitch_status stitch_pipe_create(stitch_plan* plan, int32_t depth, void* workspace, size_t bytes, stitch_pipe** out) {
  if (!plan || !out) return fail(STITCH_E_NULL, "plan or out is NULL");
  *out = nullptr;
  if (depth < 1 || depth > 8) return fail(STITCH_E_SHAPE, "depth %d outside 1..8", depth);
  const size_t need = stitch_pipe_workspace_bytes(plan, depth);
  if (!workspace) return fail(STITCH_E_WORKSPACE, "workspace is NULL");
  if (((uintptr_t)workspace & 255) != 0) return fail(STITCH_E_WORKSPACE, "workspace is not 256-byte aligned");
  if (bytes < need) return fail(STITCH_E_WORKSPACE, "workspace has %zu bytes, the pipe needs %zu", bytes, need);
  stitch_pipe* q = new (std::nothrow) stitch_pipe;
  if (!q) return fail(STITCH_E_UNSUPPORTED, "out of host memory");
  bool bound = false;
  plan_geometry(plan, &q->n, q->fw, q->fh, &q->W, &q->H, &bound);
  if (!bound) {
    delete q;
    return fail(STITCH_E_STATE, "plan has no workspace bound");
  }
  q->plan = plan;
  q->depth = depth;
  hipError_t e = hipSuccess;
  for (hipStream_t* s : {&q->s_in, &q->s_comp, &q->s_out})
    if (e == hipSuccess) e = hipStreamCreateWithFlags(s, hipStreamNonBlocking);
  // the slots, carved from the caller's workspace
  q->frames.assign((size_t)depth * q->n, nullptr);
  q->panos.assign(depth, nullptr);
  uint8_t* top = (uint8_t*)workspace;
  for (int d = 0; d < depth; ++d) {
    for (int i = 0; i < q->n; ++i) {
      q->frames[(size_t)d * q->n + i] = top;
      top += round256((size_t)q->fw[i] * q->fh[i] * 3);
    }
    q->panos[d] = top;
    top += round256((size_t)q->W * q->H * 3);
  }
  for (auto* v : {&q->ev_in, &q->ev_comp, &q->ev_out}) {
    v->assign(depth, nullptr);
    for (int d = 0; d < depth && e == hipSuccess; ++d) e = hipEventCreateWithFlags(&(*v)[d], hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    release(q);
    return hip_fail(e, "pipe set-up");
  }
  *out = q;
  return STITCH_OK;
}

stitch_status stitch_pipe_run(stitch_pipe* q, int32_t nframes, const uint8_t* const* frames, uint8_t* const* panos) {
  if (!q) return fail(STITCH_E_NULL, "pipe is NULL");
  if (nframes < 0) return fail(STITCH_E_SHAPE, "nframes %d is negative", nframes);
  if (nframes == 0) return STITCH_OK;
  if (!frames || !panos) return fail(STITCH_E_NULL, "frames or panos is NULL");
  for (int64_t k = 0; k < (int64_t)nframes * q->n; ++k)
    if (!frames[k]) return fail(STITCH_E_NULL, "frames[%lld] is NULL", (long long)k);
  for (int t = 0; t < nframes; ++t)
    if (!panos[t]) return fail(STITCH_E_NULL, "panos[%d] is NULL", t);
  const size_t pano_bytes = (size_t)q->W * q->H * 3;
  std::vector<stitch_image> fr(q->n);
  stitch_status st = STITCH_OK;
  hipError_t e = hipSuccess;
  for (int t = 0; t < nframes && !st && e == hipSuccess; ++t) {
    const int d = t % q->depth;
    const bool reuse = t >= q->depth;
    // in: the slot's frames are free once the stitch that read them (set t - depth) is done
    if (reuse) e = hipStreamWaitEvent(q->s_in, q->ev_comp[d], 0);
    for (int i = 0; i < q->n && e == hipSuccess; ++i)
      e = hipMemcpyAsync(q->frames[(size_t)d * q->n + i], frames[(size_t)t * q->n + i],
                         (size_t)q->fw[i] * q->fh[i] * 3, hipMemcpyHostToDevice, q->s_in);
    if (e == hipSuccess) e = hipEventRecord(q->ev_in[d], q->s_in);
    // stitch: after this set's frames arrived and the slot's previous panorama left
    if (e == hipSuccess) e = hipStreamWaitEvent(q->s_comp, q->ev_in[d], 0);
    if (e == hipSuccess && reuse) e = hipStreamWaitEvent(q->s_comp, q->ev_out[d], 0);
    if (e != hipSuccess) break;
    for (int i = 0; i < q->n; ++i) {
      std::memset(&fr[i], 0, sizeof fr[i]);
      fr[i].data = q->frames[(size_t)d * q->n + i];
      fr[i].width = q->fw[i];
      fr[i].height = q->fh[i];
      fr[i].channels = 3;
      fr[i].dtype = STITCH_U8;
      fr[i].layout = STITCH_HWC;
      fr[i].row_pitch = (int64_t)q->fw[i] * 3;
    }
    stitch_image pv;
    std::memset(&pv, 0, sizeof pv);
    pv.data = q->panos[d];
    pv.width = q->W;
    pv.height = q->H;
    pv.channels = 3;
    pv.dtype = STITCH_U8;
    pv.layout = STITCH_HWC;
    pv.row_pitch = (int64_t)q->W * 3;
    st = stitch_frame(q->plan, fr.data(), &pv, q->s_comp);
    if (st) break;
    e = hipEventRecord(q->ev_comp[d], q->s_comp);
    // out
    if (e == hipSuccess) e = hipStreamWaitEvent(q->s_out, q->ev_comp[d], 0);
    if (e == hipSuccess) e = hipMemcpyAsync(panos[t], q->panos[d], pano_bytes, hipMemcpyDeviceToHost, q->s_out);
    if (e == hipSuccess) e = hipEventRecord(q->ev_out[d], q->s_out);
  }
  // drain every stream, also after an error, so no copy outlives the call
  for (hipStream_t s : {q->s_in, q->s_comp, q->s_out}) {
    const hipError_t e2 = hipStreamSynchronize(s);
    if (e == hipSuccess) e = e2;
  }
  if (st) return st;
  return e == hipSuccess ? STITCH_OK : hip_fail(e, "pipe run");
}

void stitch_pipe_destroy(stitch_pipe* q) {
  if (q) release(q);
}

stitch_status stitch_host_alloc(size_t bytes, void** out) {
  if (!out) return fail(STITCH_E_NULL, "out is NULL");
  *out = nullptr;
  const hipError_t e = hipHostMalloc(out, bytes, hipHostMallocDefault);
  if (e != hipSuccess) {
    *out = nullptr;
    return hip_fail(e, "pinned host allocation");
  }
  return STITCH_OK;
}

void stitch_host_free(void* p) {
  if (p) (void)hipHostFree(p);
}

}  // extern "C"
