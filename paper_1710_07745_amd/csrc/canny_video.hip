// Streaming integer Canny over a sequence of equally sized host frames (the
// paper's stated direction of high-resolution image and video work; the
// operator per frame is canny_u8, Section 2.2.1 Steps 1-4).
//
// A ring of `depth` device slots (input frame, edge map, workspace), each
// with its own stream: frame k goes to slot k mod depth, and its
// host-to-device copy, canny_u8 and device-to-host copy are enqueued on that
// slot's stream.  The stream orders a slot's reuse after its previous frame
// (no events, no cross-stream waits), and different slots' streams run
// concurrently, so with depth >= 3 the upload of one frame, the detection of
// another and the download of a third overlap.  A push is seven runtime calls
// (two copies and canny_u8's five launches) and returns at once; the copies
// are asynchronous when the host buffers are pinned.  Every stream is
// created at the default priority.
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
    struct Slot {
        uint8_t* in = nullptr;
        uint8_t* edges = nullptr;
        void* ws = nullptr;
        hipStream_t stream = nullptr;
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
        if (s.stream) (void)hipStreamDestroy(s.stream);
    }
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
    hipError_t e = hipSuccess;
    v->slots.resize(depth);
    for (auto& s : v->slots) {
        if (e == hipSuccess) e = hipMalloc(&s.in, frame);
        if (e == hipSuccess) e = hipMalloc(&s.edges, frame);
        if (e == hipSuccess) e = hipMalloc(&s.ws, v->ws_bytes);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking);
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
    // the slot's stream runs its previous frame's download before this upload
    if (hipMemcpyAsync(s.in, host_frame, frame, hipMemcpyHostToDevice, s.stream) != hipSuccess)
        return CANNY_ERR_HIP;
    const int st = canny_u8(s.in, v->W, v->H, v->W, v->low, v->high, s.edges, v->W, nullptr, s.ws,
                            v->ws_bytes, s.stream);
    if (st != CANNY_OK) return st;
    if (hipMemcpyAsync(host_edges, s.edges, frame, hipMemcpyDeviceToHost, s.stream) != hipSuccess)
        return CANNY_ERR_HIP;
    ++v->next;
    return CANNY_OK;
}

int canny_video_sync(canny_video* v) {
    if (!v) return CANNY_ERR_INVALID;
    hipError_t e = hipSuccess;
    for (auto& s : v->slots)
        if (e == hipSuccess) e = hipStreamSynchronize(s.stream);
    return e == hipSuccess ? CANNY_OK : CANNY_ERR_HIP;
}

void canny_video_destroy(canny_video* v) {
    if (!v) return;
    (void)canny_video_sync(v);
    release(v);
}

}  // extern "C"
