/*
 * canny.h -- C ABI of the MI355X (gfx950) Canny edge detector library
 * (libcanny.so).
 *
 * The operator is the paper's four-step pipeline (Section 2.2.1, Steps 1-4;
 * step order of Algorithm 1): noise filter, Sobel gradient strength and
 * direction, non-maximum suppression, and hysteresis with a lower and an
 * upper threshold.  The readings of what the paper leaves open are fixed
 * here and stated per call: replicate (clamp-to-edge) borders at every
 * stage, ties in non-maximum suppression go to the earlier pixel in raster
 * order, strong = strength > high, weak = low <= strength <= high,
 * 8-connected hysteresis through weak pixels.
 *
 * Conventions for every call:
 *  - Pointers are DEVICE pointers owned by the caller unless marked "host".
 *    The library never frees, reallocates or retains them past the call.
 *  - Images are row-major with a row pitch given in ELEMENTS (bytes for
 *    uint8 images, floats for float images); pitch >= W.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Every call only
 *    enqueues work on `stream` and returns; results are valid once the
 *    stream has been synchronised.  No call synchronises the host.
 *  - Arguments are validated before anything is enqueued.  On an invalid
 *    argument the call returns CANNY_ERR_INVALID (too-small workspace:
 *    CANNY_ERR_WORKSPACE) and writes nothing.  A launch failure reported by
 *    the HIP runtime returns CANNY_ERR_HIP.  No C++ exception crosses the ABI.
 *  - Calls on different streams with distinct workspaces may overlap.
 *  - Class map ("class2"): 2 bits per pixel, 4 pixels per byte, pixel x of a
 *    row at bits 2*(x%4)..2*(x%4)+1 of byte x/4 (LSB first); codes 0 = none,
 *    1 = weak, 2 = strong.  Row pitch is canny_class_pitch(W) bytes.  Bits of
 *    pixels x >= W in the last byte of a row are 0; padding bytes past
 *    ceil(W/4) are unspecified.
 *  - Edge maps are uint8: 255 on an edge pixel, 0 elsewhere.
 */
#ifndef CANNY_H
#define CANNY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    CANNY_OK = 0,
    CANNY_ERR_INVALID = 1,     /* bad argument; nothing enqueued        */
    CANNY_ERR_WORKSPACE = 2,   /* workspace missing or too small        */
    CANNY_ERR_HIP = 3,         /* the HIP runtime reported an error      */
    CANNY_ERR_UNSUPPORTED = 4, /* device is not gfx950                  */
    CANNY_ERR_TOO_LARGE = 5    /* canny_u8_noalloc: image needs more than
                                  CANNY_NOALLOC_SCRATCH_BYTES of scratch */
};

/* Human-readable name of a status code (static string, never NULL). */
const char* canny_status_string(int status);

/* Library ABI version (incremented on any signature or enum change). */
int canny_abi_version(void);

/* Row pitch in bytes of the 2-bit class map for width W:
 * ceil(W/4) rounded up to a multiple of 4.  Returns 0 if W < 1. */
int64_t canny_class_pitch(int W);

/* ---------------------------------------------------------------------
 * Integer Canny (Steps 1-4 on uint8 images).
 *
 * Step 1: 5x5 binomial filter, weights (1,4,6,4,1) per axis, one rounding
 *         of the exact sum: B = (S + 128) >> 8.
 * Step 2: Sobel pair (correlation, x right, y down) in int32,
 *         strength M = |Gx| + |Gy| (0..2040), direction = the nearest of
 *         0/45/90/135 degrees to atan2(Gy, Gx) (computed exactly in integers).
 * Step 3: keep p iff M(p) > M(p - d) and M(p) >= M(p + d), d the direction.
 * Step 4: class 2 if kept and M > high, class 1 if kept and M >= low;
 *         edge iff class >= 1 and 8-connected through class >= 1 pixels to a
 *         class-2 pixel.
 *
 * in          uint8 H x W, pitch in_pitch bytes.
 * low, high   0 <= low <= high (values above 2040 never match).
 * edges       uint8 H x W output, pitch edges_pitch bytes; may be NULL if
 *             only the class map is wanted (then Step 4's connectivity pass
 *             is skipped).
 * class2      optional class-map output (see conventions) or NULL.
 * ws          device workspace of at least canny_u8_workspace_bytes(H, W)
 *             bytes, 256-byte aligned; contents on entry are ignored.
 * Errors: NULL in, H or W < 1, pitch < W, low < 0, low > high, in aliasing
 *         an output -> CANNY_ERR_INVALID.
 */
size_t canny_u8_workspace_bytes(int H, int W);
int canny_u8(const uint8_t* in, int64_t in_pitch, int H, int W, int32_t low, int32_t high,
             uint8_t* edges, int64_t edges_pitch, uint8_t* class2, void* ws, size_t ws_bytes,
             void* stream);

/* ---------------------------------------------------------------------
 * canny_u8 without a workspace argument and without any allocation, for
 * callers that cannot allocate device memory: code being recorded into a
 * HIP graph, tight serving loops, and hosts that forbid hipMalloc.
 *
 * Same operator, arguments, outputs and validation as canny_u8, minus
 * ws / ws_bytes.  The workspace is a file-scope device array of
 * CANNY_NOALLOC_SCRATCH_BYTES bytes inside the library: one copy per GPU the
 * library runs on, loaded with the library's code and held until the process
 * ends.  The call makes no hipMalloc, hipFree or other allocating call; the
 * first call on a device looks up that device's copy (hipGetSymbolAddress).
 * Images with canny_u8_workspace_bytes(H, W) > CANNY_NOALLOC_SCRATCH_BYTES
 * return CANNY_ERR_TOO_LARGE before anything is enqueued.
 * Every call on one GPU uses that GPU's single array, and it keeps the last
 * call's contents (nothing in it needs clearing: each call writes what it
 * reads).  Calls that can overlap on one GPU (different streams, or threads)
 * race on it and give wrong results; serialise them.
 */
#define CANNY_NOALLOC_SCRATCH_BYTES (32u << 20)
int canny_u8_noalloc(const uint8_t* in, int64_t in_pitch, int H, int W, int32_t low, int32_t high,
                     uint8_t* edges, int64_t edges_pitch, uint8_t* class2, void* stream);

/* ---------------------------------------------------------------------
 * Hysteresis alone (Step 4 connectivity) on a caller-provided class map.
 *
 * class2      packed class map (see conventions), pitch canny_class_pitch(W),
 *             4-byte aligned; bits of pixels x >= W are ignored.
 * edges       uint8 H x W output (255 / 0), pitch edges_pitch bytes.
 * ws          at least canny_hysteresis_workspace_bytes(H, W) bytes.
 * An edge pixel is a class >= 1 pixel 8-connected through class >= 1 pixels
 * to a class-2 pixel.  Computed by union-find connected-component labelling;
 * the result does not depend on the order of work.
 */
size_t canny_hysteresis_workspace_bytes(int H, int W);
int canny_hysteresis(const uint8_t* class2, int H, int W, uint8_t* edges, int64_t edges_pitch,
                     void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------
 * Float Canny (Steps 1-4 on fp32 images, fp32 arithmetic).
 *
 * Step 1: Gaussian filter, taps k = -radius..radius sampled from
 *         exp(-k^2 / (2 sigma^2)) and normalised to sum 1 (separable).
 * Step 2: Sobel pair, strength M = sqrt(Gx^2 + Gy^2).
 * Step 3: continuous-direction suppression: M is compared with the two
 *         values interpolated linearly on the ring of the 3x3 neighbourhood
 *         where the gradient line leaves it; keep iff M > back and
 *         M >= forward (forward = the side whose dominant-axis step is
 *         positive); M = 0 is never kept.
 * Step 4: thresholds low/high (if relative != 0, multiplied on the device
 *         by the image's largest M before suppression), classes and
 *         hysteresis as in the integer path.
 *
 * in          float H x W, pitch in_pitch floats; values must be finite.
 * sigma > 0, 1 <= radius <= 8, 0 <= low <= high.
 * With relative thresholds or max_out, the strength is first stored to the
 * workspace with its suppression decision and classified by a second,
 * elementwise pass; otherwise one kernel classifies directly.
 * edges       uint8 output or NULL (class map only).
 * class2      optional class-map output or NULL.
 * mag_out     optional float H x W strength output (pitch W) or NULL.
 * max_out     optional device float receiving the largest M, or NULL.
 * ws          at least canny_f32_workspace_bytes(H, W) bytes.
 */
size_t canny_f32_workspace_bytes(int H, int W);
int canny_f32(const float* in, int64_t in_pitch, int H, int W, float sigma, int radius,
              float low, float high, int relative, uint8_t* edges, int64_t edges_pitch,
              uint8_t* class2, float* mag_out, float* max_out, void* ws, size_t ws_bytes,
              void* stream);

/* ---------------------------------------------------------------------
 * Float Canny with the four-sector direction (Steps 1-4, fp32).
 *
 * As canny_f32 with absolute thresholds, except Step 3: the gradient
 * direction is quantised to the nearest multiple of 45 degrees (Algorithm 1
 * forms an explicit direction angle; the four sectors are those of the
 * integer path: |Gy| < tan(22.5) |Gx| -> x axis, |Gy| > tan(67.5) |Gx| ->
 * y axis, otherwise the diagonal (1, 1) when Gx and Gy share a sign, else
 * (1, -1)), and M is kept iff M > 0, M > M(p - d) and M >= M(p + d) with
 * clamped neighbours.  One kernel classifies; then hysteresis.
 * Arguments, layouts, ownership and errors as canny_f32 (low/high are
 * absolute strengths; there is no largest-strength output).
 */
int canny_f32_sector(const float* in, int64_t in_pitch, int H, int W, float sigma, int radius,
                     float low, float high, uint8_t* edges, int64_t edges_pitch, uint8_t* class2,
                     float* mag_out, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------
 * Laplacian zero-crossing detector on uint8 images (the Laplace operator
 * Laplace(f) = f_xx + f_yy that the paper's introduction names as the
 * detector Canny is compared against), after the integer path's Step 1.
 *
 * B = the 5x5 binomial filter of canny_u8 (one rounding, replicate border);
 * L = B(y,x-1) + B(y,x+1) + B(y-1,x) + B(y+1,x) - 4 B(y,x) (clamped reads);
 * an edge pixel is
 *   (a) the one nearer the zero (smaller |L|; the earlier pixel in raster
 *       order on a tie) of two 4-neighbours inside the image whose L have
 *       strictly opposite signs and |L(p) - L(q)| >= t, or
 *   (b) a pixel with L = 0 whose left and right, or upper and lower,
 *       neighbours (inside the image) have strictly opposite signs with a
 *       difference >= t.
 * One kernel; no workspace.
 *
 * in          uint8 H x W, pitch in_pitch bytes.
 * t           slope threshold >= 0 (values above 2040 give no edges).
 * edges       uint8 H x W output (255 / 0), pitch edges_pitch bytes.
 * lap         optional int16 H x W output of L (pitch lap_pitch elements,
 *             2-byte aligned) or NULL.
 * Errors: NULL in or edges, H or W outside 1..2^20, a pitch < W, t < 0,
 *         overlapping buffers -> CANNY_ERR_INVALID.
 */
int canny_log_u8(const uint8_t* in, int64_t in_pitch, int H, int W, int32_t t, uint8_t* edges,
                 int64_t edges_pitch, int16_t* lap, int64_t lap_pitch, void* stream);

/* ---------------------------------------------------------------------
 * Batched integer Canny over many images of uneven sizes.
 *
 * The same operator as canny_u8, applied to n independent images.  The
 * plan fixes the image sizes and thresholds, picks tile shapes (from an
 * on-disk autotune cache, by timing candidates when autotune != 0, else a
 * default), and records one HIP graph whose kernels each cover every tile
 * of every image in a single flat launch (one wave per forward task, one
 * workgroup per hysteresis tile, one thread per border pixel or slot).
 * canny_batch writes the per-image pointer table to the device and replays
 * the graph on `stream`.
 *
 * canny_batch_plan_create: n >= 1; H, W host arrays of n sizes (>= 1 each);
 *   0 <= low <= high; *out receives a host-owned plan.  May allocate device
 *   memory (owned by the plan) and, with autotune != 0, run timing launches
 *   on the current device; it synchronises the device.
 * canny_batch_workspace_bytes: workspace canny_batch needs.
 * canny_batch: in / edges are HOST arrays of n device pointers, in_pitch /
 *   edges_pitch HOST arrays of n pitches (bytes).  Returns
 *   CANNY_ERR_INVALID on NULL or pitch < W.  Calls with the same plan must
 *   not overlap (the plan's pointer table and graph are shared).
 * canny_batch_plan_info: host copies of the chosen forward tile height
 *   (output rows per wave) and of the hysteresis tile height.
 */
typedef struct canny_batch_plan canny_batch_plan;
int canny_batch_plan_create(int n, const int32_t* H, const int32_t* W, int32_t low, int32_t high,
                            int autotune, canny_batch_plan** out);
size_t canny_batch_workspace_bytes(const canny_batch_plan* plan);
int canny_batch(canny_batch_plan* plan, const uint8_t* const* in, const int64_t* in_pitch,
                uint8_t* const* edges, const int64_t* edges_pitch, void* ws, size_t ws_bytes,
                void* stream);
int canny_batch_plan_info(const canny_batch_plan* plan, int32_t* fwd_rows, int32_t* hyst_rows);
void canny_batch_plan_destroy(canny_batch_plan* plan);

/* ---------------------------------------------------------------------
 * Streaming integer Canny over a sequence of host frames of one size (the
 * operator of canny_u8, Steps 1-4, per frame).
 *
 * The stream owns `depth` device slots (frame, edge map, workspace), each
 * with its own HIP stream (default priority).  A push enqueues, on the next
 * slot's stream in ring order: the host-to-device copy of the frame,
 * canny_u8 on it, and the device-to-host copy of the edge map.  The slot's
 * stream orders its reuse after its previous frame; the slots' streams run
 * concurrently, so with depth >= 3 copies in both directions overlap the
 * detection.  Frames may complete out of order; canny_video_sync waits for
 * all of them.
 *
 * canny_video_create: H, W as canny_u8 accepts them (1 <= H, W <= 2^20 and
 *   ceil(H/64) * ceil(W/64) * 4096 < 2^31), 0 <= low <= high,
 *   1 <= depth <= 16; *out receives a host-owned handle.  Allocates device
 *   memory and streams (owned by the handle).  Errors: CANNY_ERR_INVALID,
 *   CANNY_ERR_UNSUPPORTED (device is not gfx950), CANNY_ERR_HIP.
 * canny_video_push: host_frame (H x W uint8, row pitch W) and host_edges
 *   (H x W uint8 output, 255 / 0) are HOST pointers; they must stay valid
 *   and unmodified (frame) / unread (edges) until canny_video_sync returns.
 *   Copies are asynchronous only for pinned host memory (hipHostMalloc);
 *   pageable memory works but the runtime may stage it synchronously.
 *   Returns at once; errors: CANNY_ERR_INVALID on NULL, CANNY_ERR_HIP.
 * canny_video_sync: waits until every pushed frame's edge map is in host
 *   memory.
 * canny_video_destroy: waits, then frees the handle.  Not thread-safe: one
 *   host thread per handle.
 */
typedef struct canny_video canny_video;
int canny_video_create(int H, int W, int32_t low, int32_t high, int depth, canny_video** out);
int canny_video_push(canny_video* v, const uint8_t* host_frame, uint8_t* host_edges);
int canny_video_sync(canny_video* v);
void canny_video_destroy(canny_video* v);

/* ---------------------------------------------------------------------
 * Differentiable front end M(I, sigma) = |Sobel * G_sigma * I| (Steps 1-2,
 * L2 strength), batched over N images of equal size, one sigma per image.
 *
 * canny_mag_forward: I float [N][H][W] contiguous, sigma float [N] (device),
 *   radius 1..12 fixed for all images (the taps are renormalised per
 *   sigma), M float [N][H][W] output.
 * canny_mag_backward: given dM = dL/dM [N][H][W], writes dL/dI
 *   [N][H][W] and dL/dsigma [N].  Replicate borders make each transposed
 *   stencil fold onto the edge pixels; dM/dG is taken as 0 where M = 0.  The
 *   blurred image is recomputed, not stored.  dsigma is reduced in a fixed
 *   order (run-to-run identical).  ws: canny_mag_backward_workspace_bytes.
 * Errors: NULL pointers, N, H, W < 1, radius outside 1..12 ->
 *   CANNY_ERR_INVALID.  sigma values are read on the device; a sigma <= 0
 *   gives unspecified output (no fault).
 */
int canny_mag_forward(const float* I, const float* sigma, int N, int H, int W, int radius,
                      float* M, void* stream);
size_t canny_mag_backward_workspace_bytes(int N, int H, int W, int radius);
int canny_mag_backward(const float* I, const float* sigma, const float* dM, int N, int H, int W,
                       int radius, float* dI, float* dsigma, void* ws, size_t ws_bytes,
                       void* stream);

/* ---------------------------------------------------------------------
 * Stage timing (diagnostics; not part of the paper's operator).
 *
 * canny_timing_begin(capacity): 1 <= capacity <= 65536.  Creates
 *   2 * capacity HIP events per stage on the current device (host-side
 *   objects, no device memory), discards earlier records, and from then on
 *   every call that runs a stage records one event before and one after that
 *   stage's kernels on the call's stream, for the first `capacity` launches
 *   of each stage.  The interval between the two events includes the
 *   launch gaps of the stage's kernels.  Do not enable it while a stream is
 *   being captured into a graph.
 * canny_timing_read(stage, ms_total, launches): host outputs; waits for the
 *   recorded events of `stage` and returns the summed milliseconds and the
 *   number of recorded launches.
 * canny_timing_end(): stops recording and destroys the events.
 * Stages: CANNY_STAGE_U8_FORWARD (canny_u8 Steps 1-3 + thresholds),
 *   CANNY_STAGE_F32_CLEAR (canny_f32: the one-thread launch that clears the
 *   largest-strength word before the walk),
 *   CANNY_STAGE_F32_WALK (canny_f32 Steps 1-3: the blur/Sobel/suppression
 *   kernel), CANNY_STAGE_F32_CLASSIFY (canny_f32 thresholds pass),
 *   CANNY_STAGE_HYSTERESIS (all hysteresis kernels of canny_u8, canny_f32,
 *   canny_hysteresis), CANNY_STAGE_MAG_FORWARD, CANNY_STAGE_MAG_BACKWARD.
 * Errors: capacity or stage out of range / NULL outputs ->
 *   CANNY_ERR_INVALID; event creation or wait failure -> CANNY_ERR_HIP.
 *   Thread-safe.
 */
enum {
    CANNY_STAGE_U8_FORWARD = 0,
    CANNY_STAGE_F32_CLEAR = 1,
    CANNY_STAGE_F32_WALK = 2,
    CANNY_STAGE_F32_CLASSIFY = 3,
    CANNY_STAGE_HYSTERESIS = 4,
    CANNY_STAGE_MAG_FORWARD = 5,
    CANNY_STAGE_MAG_BACKWARD = 6,
    CANNY_STAGE_COUNT = 7
};
int canny_timing_begin(int capacity);
int canny_timing_read(int stage, double* ms_total, int64_t* launches);
int canny_timing_end(void);

#ifdef __cplusplus
}
#endif

#endif /* CANNY_H */
