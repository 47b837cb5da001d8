// Shared pieces of the fp32 strip walks (Canny float forward and the
// differentiable front end): a lane holds 4 adjacent columns of a row.
#pragma once

#include "canny_internal.h"

namespace canny {
namespace {

struct F4 { float v[4]; };

// The lane's 4 values of a row with its columns clamped into the image, as
// four element loads through a buffer descriptor (row base in scalar
// registers): the same instructions in every lane, so that the compiler
// knows how many memory operations are outstanding and waits only for the
// row it needs.  row must be wave-uniform.
__device__ __forceinline__ F4 load_row_clamped(const float* row, int c0, int W) {
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(row), (short)0, 0x7fffffff, 0x00020000);
    F4 r;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        r.v[k] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, min(max(c0 + k, 0), W - 1) * 4, 0, 0));
    return r;
}

// The lane's 4 values of a (wave-uniform) row where ok[k] holds and 0
// elsewhere: the others are loaded from an offset past the descriptor's range,
// which reads as 0, so no select (and no wait) follows the loads.
__device__ __forceinline__ F4 load_row_masked(const float* row, int c0, const bool* ok) {
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(row), (short)0, 0x7fffffff, 0x00020000);
    F4 r;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        r.v[k] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, ok[k] ? (c0 + k) * 4 : (int)0x80000000, 0, 0));
    return r;
}

// Stores x.v[k] at column c0 + k of a (wave-uniform) row where ok[k] holds;
// the other elements get an offset past the descriptor's range and the
// hardware drops them (no branch around the stores).
__device__ __forceinline__ void store_row_masked(float* row, int c0, const F4& x, const bool* ok) {
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(row, (short)0, 0x7fffffff, 0x00020000);
#pragma unroll
    for (int k = 0; k < 4; ++k)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, x.v[k]), rs,
                                              ok[k] ? (c0 + k) * 4 : (int)0x80000000, 0, 0);
}

// value of a strip row at column offset e (relative to the lane's c0), for
// e in [-16, 19]: own 4 values, up to 4 lanes to the left or right
__device__ __forceinline__ float lane_ext(const F4& x, int e) {
    if (e >= 0 && e < 4) return x.v[e];
    if (e < 0) {
        const int hops = (-e + 3) / 4;  // lanes to the left
        float v = x.v[e + 4 * hops];
        for (int h = 0; h < hops; ++h) v = from_left_f(v);
        return v;
    }
    const int hops = e / 4;  // lanes to the right
    float v = x.v[e - 4 * hops];
    for (int h = 0; h < hops; ++h) v = from_right_f(v);
    return v;
}

// float <-> unsigned code with the same order (for atomicMin / atomicMax)
__device__ __forceinline__ uint32_t f2ord(float f) {
    const uint32_t b = bc<uint32_t>(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float ord2f(uint32_t o) {
    return bc<float>((o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o);
}

__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fminf(v, __shfl_xor(v, off));
    return v;
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
    return v;
}

struct BorderF {
    bool left, right;
    int l0_lane;
    int lw_lane, lw_px;
    bool outL[4], outR[4];
};

__device__ __forceinline__ void fix_cols(F4& x, const BorderF& bd) {
    if (bd.left) {
        const float v = bc<float>(__builtin_amdgcn_readlane(bc<int>(x.v[0]), bd.l0_lane));
#pragma unroll
        for (int k = 0; k < 4; ++k) x.v[k] = bd.outL[k] ? v : x.v[k];
    }
    if (bd.right) {
        // explicit selects on the wave-uniform lw_px: a dynamic index into x
        // would make the compiler stage the row through LDS
        const float src = bd.lw_px == 0 ? x.v[0]
                        : bd.lw_px == 1 ? x.v[1]
                        : bd.lw_px == 2 ? x.v[2] : x.v[3];
        const float v = bc<float>(__builtin_amdgcn_readlane(bc<int>(src), bd.lw_lane));
#pragma unroll
        for (int k = 0; k < 4; ++k) x.v[k] = bd.outR[k] ? v : x.v[k];
    }
}

__device__ __forceinline__ F4 sel4(bool p, const F4& a, const F4& b) {
    F4 r;
#pragma unroll
    for (int k = 0; k < 4; ++k) r.v[k] = p ? a.v[k] : b.v[k];
    return r;
}
}  // namespace
}  // namespace canny
