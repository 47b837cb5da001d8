// Internal declarations shared by the HIP translation units of libcanny.
// Device helpers (packed 16-bit arithmetic, cross-lane moves) and the host
// launchers each kernel file exports to the ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace canny {

// ---------------------------------------------------------------- constants
constexpr int kWave = 64;
constexpr int kWavesPerWG = 4;
constexpr int kWGThreads = kWave * kWavesPerWG;

// Integer forward: one wave covers 64 lanes x 4 pixels; lanes 0 and 63 carry
// the 4-pixel halo (2 blur + 1 Sobel + 1 suppression), so 62 lanes produce.
constexpr int kU8StripCols = 62 * 4;  // 248 output columns per wave

// Hysteresis tile: 64 columns (16 class-map bytes) x kHystRows rows.
constexpr int kHystCols = 64;

// ---------------------------------------------------------------- helpers
template <typename To, typename From>
__device__ __forceinline__ To bc(From v) { return __builtin_bit_cast(To, v); }

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
typedef short i16x2 __attribute__((ext_vector_type(2)));

__host__ __device__ constexpr inline int ceil_div(int a, int b) { return (a + b - 1) / b; }
__host__ __device__ constexpr inline int64_t ceil_div64(int64_t a, int64_t b) { return (a + b - 1) / b; }

// lane i receives lane i-1's value (lane 0 receives 0)
__device__ __forceinline__ uint32_t from_left(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x138, 0xF, 0xF, true);
}
// lane i receives lane i+1's value (lane 63 receives 0)
__device__ __forceinline__ uint32_t from_right(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x130, 0xF, 0xF, true);
}
__device__ __forceinline__ float from_left_f(float v) { return bc<float>(from_left(bc<uint32_t>(v))); }
__device__ __forceinline__ float from_right_f(float v) { return bc<float>(from_right(bc<uint32_t>(v))); }

// Workgroup index remapped so that each XCD (8 per chip, fed round-robin)
// walks a contiguous range of logical workgroups.
__device__ __forceinline__ int xcd_remap(int wg, int nwg) {
    const int per = (nwg + 7) >> 3;
    const int xcd = wg & 7;
    const int idx = wg >> 3;
    // the first (nwg % 8) XCDs get `per` groups, the rest `per - 1`
    const int rem = nwg & 7;
    const int full = rem == 0 ? 8 : rem;
    const int base = xcd < full ? xcd * per : full * per + (xcd - full) * (per - 1);
    return base + idx;
}

// --------------------------------------------------------------- launchers
struct U8FwdArgs {
    const uint8_t* in;
    int64_t pitch;
    int H, W;
    int low, high;  // clamped to the 16-bit range by the caller
    uint8_t* cls;
    int64_t cpitch;
};
hipError_t launch_u8_forward(const U8FwdArgs& a, int rows_per_wave, hipStream_t s);
int u8_forward_supported_rows(int rows);

struct HystArgs {
    const uint8_t* cls;
    int64_t cpitch;
    // Alternative source (float path, cls unused): the signed strength map of
    // the float walk, classified on the fly with the thresholds below (scaled
    // by the largest strength in maxbits when relative); the largest
    // strength is also written to max_out when that is non-NULL.
    const float* smag = nullptr;
    int64_t spitch = 0;
    const uint32_t* maxbits = nullptr;
    float low = 0.0f, high = 0.0f;
    int relative = 0;
    float* max_out = nullptr;
    const uint32_t* maxslots = nullptr;  // if set: the largest strength is the max of nslots
    int nslots = 0;                      // per-wave slots (16-byte aligned, <= kMaxSlots; maxbits unused)
    int H, W;
    uint8_t* edges;
    int64_t epitch;
    int32_t* blab;    // [ntiles * perim] union-find key of each border pixel's component
                      // (name tile * 256 + border index, plus 2^30 if weak; -1: none)
    int32_t* parent;  // [ntiles * 256] union-find forest over keys, indexed by name
    uint64_t* pmask;  // [ntiles * 4] per wave of a tile: which thread segments hold pending codes
};
int hyst_tile_rows_default();
size_t hyst_workspace_bytes(int H, int W, int tile_rows);
void hyst_carve(void* ws, int H, int W, int tile_rows, HystArgs& a);
hipError_t launch_hysteresis(const HystArgs& a, int tile_rows, hipStream_t s);

struct F32FwdArgs {
    const float* in;
    int64_t pitch;
    int H, W;
    float g[17];  // taps 0..radius (symmetric)
    int radius;
    float low, high;
    int relative;
    uint32_t* maxbits;  // device word: float bits of the largest M (>= 0)
    float* smag;        // signed strength map (+M kept, -M suppressed) or NULL for
    int64_t spitch;     // the one-launch absolute path; pitch in floats, multiple of 4
    uint8_t* cls;
    int64_t cpitch;
    float* mag;       // optional
    float* max_out;   // optional
    int skip_classify;  // signed path only: the hysteresis pass classifies instead
    int sector;         // one-launch path only: four-sector direction instead of interpolation
    uint32_t* maxslots = nullptr;  // signed path: one largest-M slot per wave (no clearing) instead of maxbits
};
// Largest number of per-wave maximum slots the float workspace holds; the
// hysteresis local pass reduces them in every workgroup.
constexpr int kMaxSlots = 4096;
int f32_walk_waves(const F32FwdArgs& a);  // waves of the walk launch for a
// Laplacian zero-crossing detector (canny_log.hip)
struct LogArgs {
    const uint8_t* in;
    int64_t pitch;
    int H, W;
    int t;          // slope threshold, clamped to 0..2041 by the caller
    uint8_t* edges;
    int64_t epitch;
    int estore4;    // edges 4-byte aligned with a pitch multiple of 4
    int16_t* lap;   // optional Laplacian output or NULL
    int64_t lpitch; // in elements
};
hipError_t launch_log_u8(const LogArgs& a, hipStream_t s);

// stage timing (canny_timing.hip): timing_begin returns a slot (or -1 when
// timing is off or the stage's pool is full) that timing_end closes
int timing_begin(int stage, hipStream_t s);
void timing_end(int stage, int slot, hipStream_t s);
struct StageTimer {
    int stage, slot;
    hipStream_t s;
    StageTimer(int st, hipStream_t st_s) : stage(st), slot(timing_begin(st, st_s)), s(st_s) {}
    ~StageTimer() { timing_end(stage, slot, s); }
    StageTimer(const StageTimer&) = delete;
    StageTimer& operator=(const StageTimer&) = delete;
};

hipError_t launch_f32_forward(const F32FwdArgs& a, hipStream_t s);

// ---------------------------------------------------------------- batches
// Per-image descriptor of a batch plan (device copy rewritten by every call:
// caller pointers change, the layout does not).
struct BatchImage {
    const uint8_t* in;
    int64_t pitch;
    uint8_t* edges;
    int64_t epitch;
    int H, W;
    int64_t cpitch;
    int64_t cls_off, blab_off, parent_off, pmask_off;  // bytes into the workspace
    int fwd_strips_x, fwd_base;  // forward wave tasks before this image
    int tiles_x, tiles_y, tile_base;
    int merge_base;
};
struct BatchDev {
    char* ws;
    const int32_t* tile_img;  // image index of every tile of the batch (tile_base order)
    int n;
    int low, high;
    int total_fwd, total_tiles, total_merge;
};
hipError_t launch_u8_forward_batch(const BatchImage* imgs, const BatchDev* hdr, int rows_per_wave,
                                   int total_fwd, hipStream_t s);
hipError_t launch_hyst_batch(const BatchImage* imgs, const BatchDev* hdr, int total_tiles,
                             int total_merge, hipStream_t s);

size_t mag_partials(int N, int H, int W, int radius);
hipError_t launch_mag_forward(const float* I, const float* sigma, int N, int H, int W, int radius,
                              float* M, hipStream_t s);
hipError_t launch_mag_backward(const float* I, const float* sigma, const float* dM, int N, int H, int W,
                               int radius, float* dI, float* dsigma, float* dB, float* partial,
                               hipStream_t s);

}  // namespace canny
