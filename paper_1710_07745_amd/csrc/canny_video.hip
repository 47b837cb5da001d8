// Streaming integer Canny over a sequence of equally sized host frames (the
// paper's stated direction of high-resolution image and video work; the
// operator per frame is canny_u8, Section 2.2.1 Steps 1-4).
//
// A ring of `depth` device slots (input frame, edge map, workspace) and three
// streams: frame k is copied host-to-device on the upload stream, detected on
// the compute stream after the upload's event, and its edge map copied back on
// the download stream after the detection's event.  A slot is reused only
// after its previous download has finished (the upload waits on that event),
// so with depth >= 3 the upload of frame k+1, the detection of frame k and the
// download of frame k-1 run at the same time.  All waits are device-side; a
// push returns at once (the copies are asynchronous when the host buffers are
// pinned).  Every stream is created at the default priority.
#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/canny.h"

namespace canny {
bool device_ok();
bool size_ok(int H, int W);
}  // namespace canny

struct canny_video {
    int H = 0, W = 0, depth = 0;
    int32_t low = 0, high = 0;
    size_t ws_bytes = 0;
    hipStream_t up = nullptr, comp = nullptr, down = nullptr;
    struct Slot {
        uint8_t* in = nullptr;
        uint8_t* edges = nullptr;
        void* ws = nullptr;
        hipEvent_t uploaded = nullptr, detected = nullptr, downloaded = nullptr;
        bool used = false;
    };
    std::vector<Slot> slots;
    int64_t next = 0;
};

namespace {

constexpr int kMaxDepth = 16;

void release(canny_video* v) {
    if (!v) return;
    for (auto& s : v->slots) {
        if (s.in) (void)hipFree(s.in);
        if (s.edges) (void)hipFree(s.edges);
        if (s.ws) (void)hipFree(s.ws);
        if (s.uploaded) (void)hipEventDestroy(s.uploaded);
        if (s.detected) (void)hipEventDestroy(s.detected);
        if (s.downloaded) (void)hipEventDestroy(s.downloaded);
    }
    if (v->up) (void)hipStreamDestroy(v->up);
    if (v->comp) (void)hipStreamDestroy(v->comp);
    if (v->down) (void)hipStreamDestroy(v->down);
    delete v;
}

}  // namespace

extern "C" {

int canny_video_create(int H, int W, int32_t low, int32_t high, int depth, canny_video** out) {
    // the frame sizes canny_u8 accepts (each side <= 2^20, and the hysteresis
    // tile bound), checked here so that no push can fail on the size
    if (!out || !canny::size_ok(H, W) || low < 0 || low > high || depth < 1 || depth > kMaxDepth)
        return CANNY_ERR_INVALID;
    *out = nullptr;
    if (!canny::device_ok()) return CANNY_ERR_UNSUPPORTED;
    canny_video* v = new canny_video();
    v->H = H;
    v->W = W;
    v->depth = depth;
    v->low = low;
    v->high = high;
    v->ws_bytes = canny_u8_workspace_bytes(H, W);
    const size_t frame = (size_t)H * W;
    hipError_t e = hipStreamCreateWithFlags(&v->up, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&v->comp, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&v->down, hipStreamNonBlocking);
    v->slots.resize(depth);
    for (auto& s : v->slots) {
        if (e == hipSuccess) e = hipMalloc(&s.in, frame);
        if (e == hipSuccess) e = hipMalloc(&s.edges, frame);
        if (e == hipSuccess) e = hipMalloc(&s.ws, v->ws_bytes);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s.uploaded, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s.detected, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s.downloaded, hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        release(v);
        return CANNY_ERR_HIP;
    }
    *out = v;
    return CANNY_OK;
}

int canny_video_push(canny_video* v, const uint8_t* host_frame, uint8_t* host_edges) {
    if (!v || !host_frame || !host_edges) return CANNY_ERR_INVALID;
    canny_video::Slot& s = v->slots[(size_t)(v->next % v->depth)];
    const size_t frame = (size_t)v->H * v->W;
    hipError_t e = hipSuccess;
    // the slot's previous frame must be downloaded before its buffers are reused
    if (s.used) e = hipStreamWaitEvent(v->up, s.downloaded, 0);
    if (e == hipSuccess) e = hipMemcpyAsync(s.in, host_frame, frame, hipMemcpyHostToDevice, v->up);
    if (e == hipSuccess) e = hipEventRecord(s.uploaded, v->up);
    if (e == hipSuccess) e = hipStreamWaitEvent(v->comp, s.uploaded, 0);
    if (e != hipSuccess) return CANNY_ERR_HIP;
    const int st = canny_u8(s.in, v->W, v->H, v->W, v->low, v->high, s.edges, v->W, nullptr, s.ws,
                            v->ws_bytes, v->comp);
    if (st != CANNY_OK) return st;
    e = hipEventRecord(s.detected, v->comp);
    if (e == hipSuccess) e = hipStreamWaitEvent(v->down, s.detected, 0);
    if (e == hipSuccess) e = hipMemcpyAsync(host_edges, s.edges, frame, hipMemcpyDeviceToHost, v->down);
    if (e == hipSuccess) e = hipEventRecord(s.downloaded, v->down);
    if (e != hipSuccess) return CANNY_ERR_HIP;
    s.used = true;
    ++v->next;
    return CANNY_OK;
}

int canny_video_sync(canny_video* v) {
    if (!v) return CANNY_ERR_INVALID;
    hipError_t e = hipStreamSynchronize(v->up);
    if (e == hipSuccess) e = hipStreamSynchronize(v->comp);
    if (e == hipSuccess) e = hipStreamSynchronize(v->down);
    return e == hipSuccess ? CANNY_OK : CANNY_ERR_HIP;
}

void canny_video_destroy(canny_video* v) {
    if (!v) return;
    (void)canny_video_sync(v);
    release(v);
}

}  // extern "C"
