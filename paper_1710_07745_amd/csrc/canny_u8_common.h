// Shared pieces of the uint8 strip walks (integer Canny forward and the
// Laplacian zero-crossing detector): lane l of a wave holds four adjacent
// columns as one dword, arithmetic is packed 16-bit (two pixels per VGPR),
// horizontal neighbours cross lanes by DPP shifts, and the binomial blur
// (1,4,6,4,1) per axis is the integer path's Step 1.
#pragma once

#include "canny_internal.h"

namespace canny {
namespace {

__device__ __forceinline__ u16x2 U(uint32_t v) { return bc<u16x2>(v); }
__device__ __forceinline__ i16x2 S(uint32_t v) { return bc<i16x2>(v); }
__device__ __forceinline__ uint32_t W32(u16x2 v) { return bc<uint32_t>(v); }
__device__ __forceinline__ uint32_t W32(i16x2 v) { return bc<uint32_t>(v); }
__device__ __forceinline__ uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel) {
    return __builtin_amdgcn_perm(hi, lo, sel);
}
__device__ __forceinline__ uint32_t align16(uint32_t hi, uint32_t lo) {
    return __builtin_amdgcn_alignbit(hi, lo, 16);
}
// per-bit select: m ? a : b
__device__ __forceinline__ uint32_t bsel(uint32_t m, uint32_t a, uint32_t b) {
    return (a & m) | (b & ~m);
}

// Border description of one wave strip (all fields wave-uniform except masks).
struct Border {
    bool left, right;       // strip touches column 0 / column W-1
    int l0_lane;            // lane holding column 0
    int lw_lane, lw_pair;   // lane and pair holding column W-1
    int lw_shift;           // 0 or 16
    uint32_t mL0, mL1;      // 16-bit halves whose column < 0
    uint32_t mR0, mR1;      // 16-bit halves whose column >= W
};

// Replicate the edge column into halves outside the image.
__device__ __forceinline__ void fix_cols(uint32_t& p0, uint32_t& p1, const Border& bd) {
    if (bd.left) {
        uint32_t v = (uint32_t)__builtin_amdgcn_readlane((int)p0, bd.l0_lane);
        v = (v & 0xFFFFu) * 0x10001u;
        p0 = bsel(bd.mL0, v, p0);
        p1 = bsel(bd.mL1, v, p1);
    }
    if (bd.right) {
        uint32_t src = bd.lw_pair ? p1 : p0;
        uint32_t v = (uint32_t)__builtin_amdgcn_readlane((int)src, bd.lw_lane);
        v = ((v >> bd.lw_shift) & 0xFFFFu) * 0x10001u;
        p0 = bsel(bd.mR0, v, p0);
        p1 = bsel(bd.mR1, v, p1);
    }
}

// The lane's 4 pixels with replicated borders as four byte loads: the same
// instructions in every lane (no branch), so the walk's load-wait counts stay
// exact.
__device__ __forceinline__ uint32_t load_px4_clamped(const uint8_t* row, int c0, int W) {
    uint32_t v = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int c = min(max(c0 + k, 0), W - 1);
        v |= (uint32_t)row[c] << (8 * k);
    }
    return v;
}

// Horizontal 5-tap binomial of the lane's 4 pixels (needs 2 from each side).
__device__ __forceinline__ void hblur(uint32_t d, uint32_t& h0, uint32_t& h1) {
    const uint32_t dl = from_left(d), dr = from_right(d);
    const u16x2 Em1 = U(perm(0u, dl, 0x0C030C02u));  // (c0-2, c0-1)
    const u16x2 E0 = U(perm(0u, d, 0x0C010C00u));    // (c0,   c0+1)
    const u16x2 E1 = U(perm(0u, d, 0x0C030C02u));    // (c0+2, c0+3)
    const u16x2 E2 = U(perm(0u, dr, 0x0C010C00u));   // (c0+4, c0+5)
    const u16x2 Om1 = U(perm(d, dl, 0x0C040C03u));   // (c0-1, c0)
    const u16x2 O0 = U(perm(0u, d, 0x0C020C01u));    // (c0+1, c0+2)
    const u16x2 O1 = U(perm(dr, d, 0x0C040C03u));    // (c0+3, c0+4)
    const u16x2 four = {4, 4}, six = {6, 6};
    h0 = W32((Em1 + E1) + (Om1 + O0) * four + E0 * six);
    h1 = W32((E0 + E2) + (O0 + O1) * four + E1 * six);
}

// Balanced single-image launch.  A border wave (clamped loads, per-stage
// replication) costs about 1.7x an interior wave per row, and with one block
// height the border waves set the kernel's end; so border blocks are RRE rows
// tall and interior blocks RRI > RRE.  Waves [0, edge_waves) walk the border
// strips ({0} and [sr, strips_x), or every strip when rows are not 4-byte
// aligned) block-major; the rest walk the interior strips [1, sr), each with
// one border block at the top, k interior blocks from row RRE, and nb border
// blocks below them.
struct U8Plan {
    int nwaves, edge_waves;
    int n_es, sr, n_is;
    int k, nb;
};


inline U8Plan make_u8_plan(int H, int W, int fast_ok, int RRI, int RRE) {
    U8Plan p{};
    const int strips_x = ceil_div(W, kU8StripCols);
    int sr = strips_x;  // first strip whose right halo leaves the image
    if (!fast_ok || strips_x == 1) {
        sr = 1;
    } else {
        for (int s = 1; s < strips_x; ++s)
            if ((int64_t)(s + 1) * kU8StripCols + 4 > W) {
                sr = s;
                break;
            }
    }
    p.sr = sr;
    p.n_es = 1 + (strips_x - sr);
    p.n_is = sr - 1;
    p.k = H >= 2 * RRE ? (H - 2 * RRE) / RRI : 0;
    p.nb = ceil_div(max(0, H - RRE - p.k * RRI), RRE);
    p.edge_waves = p.n_es * ceil_div(H, RRE);
    p.nwaves = p.edge_waves + p.n_is * (1 + p.k + p.nb);
    return p;
}

// The interior conditions the balanced kernel relies on, checked on the host
// (they hold by construction): halo rows and columns of every interior block
// inside the image, 4-byte aligned rows.
inline bool u8_plan_ok(const U8Plan& p, int H, int W, int fast_ok, int RRI, int RRE) {
    if (p.n_is == 0 || p.k == 0) return true;  // no interior block
    return fast_ok && RRE >= 4 && RRE + p.k * RRI + 4 <= H &&
           (int64_t)p.sr * kU8StripCols + 4 <= W;  // last interior strip is sr - 1
}

}  // namespace
}  // namespace canny
