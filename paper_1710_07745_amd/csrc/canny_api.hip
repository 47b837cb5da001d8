// C ABI of libcanny: argument validation, workspace layout and dispatch for
// the single-image integer and float paths.  Every check runs before any
// work is enqueued; no call synchronises the host.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>

#include "../../include/canny.h"
#include "canny_internal.h"

namespace canny {

static constexpr size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

static hipError_t timed_hysteresis(const HystArgs& h, int tile_rows, hipStream_t s) {
    StageTimer t(CANNY_STAGE_HYSTERESIS, s);
    return launch_hysteresis(h, tile_rows, s);
}

bool device_ok() {
    static std::mutex mu;
    static int cached[64];  // 0 unknown, 1 ok, 2 unsupported
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return false;
    std::lock_guard<std::mutex> lk(mu);
    if (!cached[dev]) {
        hipDeviceProp_t p;
        if (hipGetDeviceProperties(&p, dev) != hipSuccess) return false;
        cached[dev] = std::strncmp(p.gcnArchName, "gfx950", 6) == 0 ? 1 : 2;
    }
    return cached[dev] == 1;
}

// Sizes whose tile-rounded pixel count fits 31 bits (e.g. 46000 x 46000):
// pixel offsets of the tiles, and the hysteresis pass's component names
// (below 2^27) with their weak bit, stay within int32.
bool size_ok(int H, int W) {
    return H >= 1 && W >= 1 && H <= (1 << 20) && W <= (1 << 20) &&
           (int64_t)ceil_div(H, 64) * ceil_div(W, 64) * 4096 < ((int64_t)1 << 31);
}

static bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
    if (!a || !b || !na || !nb) return false;
    const char* pa = static_cast<const char*>(a);
    const char* pb = static_cast<const char*>(b);
    return pa < pb + nb && pb < pa + na;
}

static size_t image_bytes(int H, int64_t pitch, int W, size_t elem) {
    return ((size_t)(H - 1) * (size_t)pitch + (size_t)W) * elem;
}

int64_t class_pitch(int W) { return W < 1 ? 0 : ((int64_t)ceil_div(W, 4) + 3) & ~(int64_t)3; }

static size_t class_bytes(int H, int W) { return align256((size_t)H * class_pitch(W)); }

static int status_of(hipError_t e) { return e == hipSuccess ? CANNY_OK : CANNY_ERR_HIP; }

}  // namespace canny

using namespace canny;

extern "C" {

const char* canny_status_string(int status) {
    switch (status) {
        case CANNY_OK: return "ok";
        case CANNY_ERR_INVALID: return "invalid argument";
        case CANNY_ERR_WORKSPACE: return "workspace missing or too small";
        case CANNY_ERR_HIP: return "HIP runtime error";
        case CANNY_ERR_UNSUPPORTED: return "unsupported device (gfx950 required)";
        case CANNY_ERR_TOO_LARGE: return "image too large for the allocation-free entry point's scratch";
        default: return "unknown status";
    }
}

int canny_abi_version(void) { return 5; }

int64_t canny_class_pitch(int W) { return class_pitch(W); }

size_t canny_u8_workspace_bytes(int H, int W) {
    if (!size_ok(H, W)) return 0;
    return class_bytes(H, W) + hyst_workspace_bytes(H, W, hyst_tile_rows_default());
}

}  // extern "C"

namespace canny {

static bool u8_args_ok(const uint8_t* in, int64_t in_pitch, int H, int W, int32_t low, int32_t high,
                       const uint8_t* edges, int64_t edges_pitch, const uint8_t* class2) {
    if (!in || !size_ok(H, W) || in_pitch < W || low < 0 || low > high) return false;
    if (edges && edges_pitch < W) return false;
    if (class2 && ((uintptr_t)class2 % 4)) return false;
    const size_t nin = image_bytes(H, in_pitch, W, 1);
    if (edges && overlaps(in, nin, edges, image_bytes(H, edges_pitch, W, 1))) return false;
    if (class2 && overlaps(in, nin, class2, (size_t)H * class_pitch(W))) return false;
    return true;
}

// canny_u8 after validation: the forward and the hysteresis passes on the
// workspace ws (canny_u8_workspace_bytes(H, W) bytes, 256-byte aligned).
static int u8_run(const uint8_t* in, int64_t in_pitch, int H, int W, int32_t low, int32_t high,
                  uint8_t* edges, int64_t edges_pitch, uint8_t* class2, void* ws, void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* w = static_cast<char*>(ws);
    U8FwdArgs f;
    f.in = in;
    f.pitch = in_pitch;
    f.H = H;
    f.W = W;
    f.low = low > 2041 ? 2041 : low;
    f.high = high > 2040 ? 2040 : high;
    f.cls = class2 ? class2 : reinterpret_cast<uint8_t*>(w);
    f.cpitch = class_pitch(W);
    hipError_t e;
    {
        StageTimer t(CANNY_STAGE_U8_FORWARD, s);
        e = launch_u8_forward(f, 0, s);  // balanced block heights
    }
    if (e != hipSuccess || !edges) return status_of(e);
    HystArgs h;
    h.cls = f.cls;
    h.cpitch = f.cpitch;
    h.H = H;
    h.W = W;
    h.edges = edges;
    h.epitch = edges_pitch;
    const int T = hyst_tile_rows_default();
    hyst_carve(w + class_bytes(H, W), H, W, T, h);
    return status_of(timed_hysteresis(h, T, s));
}

// Scratch of canny_u8_noalloc: one array per GPU the library runs on, held
// until the process ends.  In host code `scratch` names a host-side stand-in;
// the device address comes from hipGetSymbolAddress, once per device, and is
// the only form of it that host code passes on.
static __device__ __align__(256) unsigned char scratch[CANNY_NOALLOC_SCRATCH_BYTES];

static void* scratch_address(int* status) {
    static std::mutex mu;
    static void* addr[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
        *status = CANNY_ERR_HIP;
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            *status = CANNY_ERR_HIP;
            return nullptr;
        }
        addr[dev] = p;
    }
    return addr[dev];
}

}  // namespace canny

extern "C" {

int canny_u8(const uint8_t* in, int64_t in_pitch, int H, int W, int32_t low, int32_t high,
             uint8_t* edges, int64_t edges_pitch, uint8_t* class2, void* ws, size_t ws_bytes,
             void* stream) {
    if (!u8_args_ok(in, in_pitch, H, W, low, high, edges, edges_pitch, class2)) return CANNY_ERR_INVALID;
    const size_t need = canny_u8_workspace_bytes(H, W);
    if (!ws || ws_bytes < need || ((uintptr_t)ws % 256)) return CANNY_ERR_WORKSPACE;
    if (!device_ok()) return CANNY_ERR_UNSUPPORTED;
    return u8_run(in, in_pitch, H, W, low, high, edges, edges_pitch, class2, ws, stream);
}

int canny_u8_noalloc(const uint8_t* in, int64_t in_pitch, int H, int W, int32_t low, int32_t high,
                     uint8_t* edges, int64_t edges_pitch, uint8_t* class2, void* stream) {
    if (!u8_args_ok(in, in_pitch, H, W, low, high, edges, edges_pitch, class2)) return CANNY_ERR_INVALID;
    if (canny_u8_workspace_bytes(H, W) > (size_t)CANNY_NOALLOC_SCRATCH_BYTES) return CANNY_ERR_TOO_LARGE;
    if (!device_ok()) return CANNY_ERR_UNSUPPORTED;
    int status = CANNY_OK;
    void* ws = scratch_address(&status);
    if (!ws) return status;
    // the passes write every workspace word they later read (class map,
    // border names, union-find entries of this call's components, pending
    // masks), so nothing left by an earlier call needs clearing
    return u8_run(in, in_pitch, H, W, low, high, edges, edges_pitch, class2, ws, stream);
}

size_t canny_hysteresis_workspace_bytes(int H, int W) {
    if (!size_ok(H, W)) return 0;
    return hyst_workspace_bytes(H, W, hyst_tile_rows_default());
}

int canny_hysteresis(const uint8_t* class2, int H, int W, uint8_t* edges, int64_t edges_pitch,
                     void* ws, size_t ws_bytes, void* stream) {
    if (!class2 || !edges || !size_ok(H, W) || edges_pitch < W || ((uintptr_t)class2 % 4))
        return CANNY_ERR_INVALID;
    if (overlaps(class2, (size_t)H * class_pitch(W), edges, image_bytes(H, edges_pitch, W, 1)))
        return CANNY_ERR_INVALID;
    const size_t need = canny_hysteresis_workspace_bytes(H, W);
    if (!ws || ws_bytes < need || ((uintptr_t)ws % 256)) return CANNY_ERR_WORKSPACE;
    if (!device_ok()) return CANNY_ERR_UNSUPPORTED;
    HystArgs h;
    h.cls = class2;
    h.cpitch = class_pitch(W);
    h.H = H;
    h.W = W;
    h.edges = edges;
    h.epitch = edges_pitch;
    const int T = hyst_tile_rows_default();
    hyst_carve(ws, H, W, T, h);
    return status_of(timed_hysteresis(h, T, static_cast<hipStream_t>(stream)));
}

static int64_t smag_pitch(int W) { return ((int64_t)W + 3) & ~(int64_t)3; }
// float workspace header: the largest-strength word (256 bytes), then the
// walk's per-wave largest-strength slots
static constexpr size_t kF32SlotsOff = 256;
static constexpr size_t kF32Header = kF32SlotsOff + align256(4 * (size_t)kMaxSlots);

size_t canny_f32_workspace_bytes(int H, int W) {
    if (!size_ok(H, W)) return 0;
    return kF32Header + class_bytes(H, W) + hyst_workspace_bytes(H, W, hyst_tile_rows_default()) +
           align256((size_t)H * smag_pitch(W) * 4);
}

static int f32_impl(const float* in, int64_t in_pitch, int H, int W, float sigma, int radius,
                    float low, float high, int relative, uint8_t* edges, int64_t edges_pitch,
                    uint8_t* class2, float* mag_out, float* max_out, void* ws, size_t ws_bytes,
                    void* stream, int sector) {
    if (!in || !size_ok(H, W) || in_pitch < W) return CANNY_ERR_INVALID;
    if (!(sigma > 0.0f) || !std::isfinite(sigma) || radius < 1 || radius > 8) return CANNY_ERR_INVALID;
    if (!(low >= 0.0f) || !(high >= low) || !std::isfinite(high)) return CANNY_ERR_INVALID;
    if (edges && edges_pitch < W) return CANNY_ERR_INVALID;
    if (class2 && ((uintptr_t)class2 % 4)) return CANNY_ERR_INVALID;
    const size_t nin = image_bytes(H, in_pitch, W, 4);
    if (edges && overlaps(in, nin, edges, image_bytes(H, edges_pitch, W, 1))) return CANNY_ERR_INVALID;
    if (class2 && overlaps(in, nin, class2, (size_t)H * class_pitch(W))) return CANNY_ERR_INVALID;
    if (mag_out && overlaps(in, nin, mag_out, (size_t)H * W * 4)) return CANNY_ERR_INVALID;
    const size_t need = canny_f32_workspace_bytes(H, W);
    if (!ws || ws_bytes < need || ((uintptr_t)ws % 256)) return CANNY_ERR_WORKSPACE;
    if (!device_ok()) return CANNY_ERR_UNSUPPORTED;

    hipStream_t s = static_cast<hipStream_t>(stream);
    char* w = static_cast<char*>(ws);
    F32FwdArgs f;
    std::memset(&f, 0, sizeof(f));
    f.in = in;
    f.pitch = in_pitch;
    f.H = H;
    f.W = W;
    {  // sampled Gaussian taps, normalised in double, rounded once to float
        double gd[17], sum = 0.0;
        for (int k = 0; k <= radius; ++k) {
            gd[k] = std::exp(-(double)k * k / (2.0 * (double)sigma * (double)sigma));
            sum += k ? 2.0 * gd[k] : gd[k];
        }
        for (int k = 0; k <= radius; ++k) f.g[k] = (float)(gd[k] / sum);
    }
    f.radius = radius;
    f.low = low;
    f.high = high;
    f.relative = relative ? 1 : 0;
    f.maxbits = reinterpret_cast<uint32_t*>(w);
    const size_t hyst_off = kF32Header + class_bytes(H, W);
    if (relative || max_out) {  // the walk stores signed strengths, a second pass classifies
        f.smag = reinterpret_cast<float*>(w + hyst_off +
                                          hyst_workspace_bytes(H, W, hyst_tile_rows_default()));
        f.spitch = smag_pitch(W);
    }
    f.cls = class2 ? class2 : reinterpret_cast<uint8_t*>(w + kF32Header);
    f.cpitch = class_pitch(W);
    f.mag = mag_out;
    f.max_out = max_out;
    // With the signed map and nothing but edges (and the max) asked for, the
    // hysteresis pass classifies straight from the signed map: no class map.
    const bool fused = f.smag && !class2 && !mag_out && edges;
    f.skip_classify = fused ? 1 : 0;
    f.sector = sector;
    // Fused: the walk leaves one largest-strength slot per wave and every
    // hysteresis workgroup reduces them, so no launch has to clear a shared
    // word first (up to kMaxSlots waves; larger images keep the word).
    const int nslots = fused ? f32_walk_waves(f) : 0;
    if (nslots > 0 && nslots <= kMaxSlots) f.maxslots = reinterpret_cast<uint32_t*>(w + kF32SlotsOff);
    hipError_t e = launch_f32_forward(f, s);
    if (e != hipSuccess || !edges) return status_of(e);
    HystArgs h;
    h.cls = f.cls;
    h.cpitch = f.cpitch;
    if (fused) {
        h.smag = f.smag;
        h.spitch = f.spitch;
        h.maxbits = f.maxbits;
        h.maxslots = f.maxslots;
        h.nslots = f.maxslots ? nslots : 0;
        h.low = low;
        h.high = high;
        h.relative = f.relative;
        h.max_out = max_out;
    }
    h.H = H;
    h.W = W;
    h.edges = edges;
    h.epitch = edges_pitch;
    const int T = hyst_tile_rows_default();
    hyst_carve(w + hyst_off, H, W, T, h);
    return status_of(timed_hysteresis(h, T, s));
}

int canny_f32(const float* in, int64_t in_pitch, int H, int W, float sigma, int radius, float low,
              float high, int relative, uint8_t* edges, int64_t edges_pitch, uint8_t* class2,
              float* mag_out, float* max_out, void* ws, size_t ws_bytes, void* stream) {
    return f32_impl(in, in_pitch, H, W, sigma, radius, low, high, relative, edges, edges_pitch,
                    class2, mag_out, max_out, ws, ws_bytes, stream, 0);
}

int canny_f32_sector(const float* in, int64_t in_pitch, int H, int W, float sigma, int radius,
                     float low, float high, uint8_t* edges, int64_t edges_pitch, uint8_t* class2,
                     float* mag_out, void* ws, size_t ws_bytes, void* stream) {
    // absolute thresholds and no largest-strength output: the walk classifies
    return f32_impl(in, in_pitch, H, W, sigma, radius, low, high, 0, edges, edges_pitch, class2,
                    mag_out, nullptr, ws, ws_bytes, stream, 1);
}

int canny_log_u8(const uint8_t* in, int64_t in_pitch, int H, int W, int32_t t, uint8_t* edges,
                 int64_t edges_pitch, int16_t* lap, int64_t lap_pitch, void* stream) {
    if (!in || !edges || !size_ok(H, W) || in_pitch < W || edges_pitch < W || t < 0)
        return CANNY_ERR_INVALID;
    if (lap && (lap_pitch < W || ((uintptr_t)lap % 2))) return CANNY_ERR_INVALID;
    const size_t nin = image_bytes(H, in_pitch, W, 1), ne = image_bytes(H, edges_pitch, W, 1);
    if (overlaps(in, nin, edges, ne)) return CANNY_ERR_INVALID;
    if (lap) {
        const size_t nl = image_bytes(H, lap_pitch, W, 2);
        if (overlaps(in, nin, lap, nl) || overlaps(edges, ne, lap, nl)) return CANNY_ERR_INVALID;
    }
    if (!device_ok()) return CANNY_ERR_UNSUPPORTED;
    LogArgs a;
    a.in = in;
    a.pitch = in_pitch;
    a.H = H;
    a.W = W;
    a.t = t > 2041 ? 2041 : t;  // |L(p) - L(q)| <= 2040
    a.edges = edges;
    a.epitch = edges_pitch;
    a.estore4 = ((uintptr_t)edges % 4 == 0) && (edges_pitch % 4 == 0);
    a.lap = lap;
    a.lpitch = lap_pitch;
    return status_of(launch_log_u8(a, static_cast<hipStream_t>(stream)));
}

static bool mag_args_ok(const float* I, const float* sigma, int N, int H, int W, int radius) {
    return I && sigma && N >= 1 && size_ok(H, W) && radius >= 1 && radius <= 12 &&
           (int64_t)N * H * W <= ((int64_t)1 << 34);
}

int canny_mag_forward(const float* I, const float* sigma, int N, int H, int W, int radius, float* M,
                      void* stream) {
    if (!mag_args_ok(I, sigma, N, H, W, radius) || !M) return CANNY_ERR_INVALID;
    const size_t n = (size_t)N * H * W * 4;
    if (overlaps(I, n, M, n) || overlaps(sigma, (size_t)N * 4, M, n)) return CANNY_ERR_INVALID;
    if (!device_ok()) return CANNY_ERR_UNSUPPORTED;
    StageTimer t(CANNY_STAGE_MAG_FORWARD, static_cast<hipStream_t>(stream));
    return status_of(launch_mag_forward(I, sigma, N, H, W, radius, M, static_cast<hipStream_t>(stream)));
}

size_t canny_mag_backward_workspace_bytes(int N, int H, int W, int radius) {
    if (N < 1 || !size_ok(H, W) || radius < 1 || radius > 12) return 0;
    return align256((size_t)N * H * W * 4) + align256(mag_partials(N, H, W, radius) * 4);
}

int canny_mag_backward(const float* I, const float* sigma, const float* dM, int N, int H, int W,
                       int radius, float* dI, float* dsigma, void* ws, size_t ws_bytes, void* stream) {
    if (!mag_args_ok(I, sigma, N, H, W, radius) || !dM || !dI || !dsigma) return CANNY_ERR_INVALID;
    const size_t n = (size_t)N * H * W * 4;
    if (overlaps(I, n, dI, n) || overlaps(dM, n, dI, n) || overlaps(dsigma, (size_t)N * 4, dI, n))
        return CANNY_ERR_INVALID;
    const size_t need = canny_mag_backward_workspace_bytes(N, H, W, radius);
    if (!ws || ws_bytes < need || ((uintptr_t)ws % 256)) return CANNY_ERR_WORKSPACE;
    if (!device_ok()) return CANNY_ERR_UNSUPPORTED;
    char* w = static_cast<char*>(ws);
    float* dB = reinterpret_cast<float*>(w);
    float* partial = reinterpret_cast<float*>(w + align256(n));
    StageTimer t(CANNY_STAGE_MAG_BACKWARD, static_cast<hipStream_t>(stream));
    return status_of(launch_mag_backward(I, sigma, dM, N, H, W, radius, dI, dsigma, dB, partial,
                                         static_cast<hipStream_t>(stream)));
}

}  // extern "C"
