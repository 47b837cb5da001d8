// Fused integer Canny forward for gfx950: Steps 1-3 and the double threshold
// of Step 4 (paper Section 2.2.1) in one pass over the uint8 image.
//
// Layout of the work: a wave owns a vertical strip.  Lane l holds the four
// input columns c0 = X0 - 4 + 4l .. c0 + 3 as one dword; lanes 0 and 63 carry
// the 4-column halo (2 for the blur, 1 for Sobel, 1 for suppression), so
// lanes 1..62 produce 248 output columns.  The wave walks the strip top to
// bottom; every stage keeps a sliding window of rows in registers:
//     input row -> horizontal binomial (h, 5-row window)
//               -> vertical binomial + rounding (B) -> Sobel row terms
//                  (dx = B(x+1) - B(x-1), sx = B(x-1) + 2B(x) + B(x+1), 3 rows)
//               -> Gx, Gy, M = |Gx| + |Gy|, direction masks (3 rows of M)
//               -> suppression + thresholds -> 2-bit codes, 1 byte per lane.
// Horizontal neighbours cross lanes with DPP wave shifts; all arithmetic is
// packed 16-bit (two pixels per VGPR).  Values stay in range: horizontal
// blur <= 4080, vertical blur + 128 <= 65408, |Gx|,|Gy| <= 1020, M <= 2040.
//
// Replicate borders are applied per stage: the input loads are clamped, and
// the blurred image B and the strength M are re-extended after they are
// formed (columns outside the image copy the edge column; rows outside copy
// the edge row), so each stage reads its predecessor exactly as the
// clamp-indexed definition does.
//
// Direction: the nearest multiple of 45 degrees to atan2(Gy, Gx).  For
// |Gx|, |Gy| <= 1020 the tan(22.5 deg) boundary test is exact as
// 408*|Gy| < 169*|Gx| (169/408 and 408/985 are consecutive continued-fraction
// convergents of sqrt(2)-1; no fraction with denominator <= 1020 lies
// between them), and the 67.5 deg test is the same with the axes swapped.
// Both are single v_dot2 instructions on a packed (|Gy|, |Gx|) pair.
#include "canny_internal.h"
#include "canny_u8_common.h"

namespace canny {
namespace {

// One row of strength with its column-shifted copies, per lane:
// c0 = (x, x+1), c1 = (x+2, x+3), sm1 = (x-1, x), s1 = (x+1, x+2), s3 = (x+3, x+4).
struct MRow {
    uint32_t c0, c1, sm1, s1, s3;
};
// Direction masks of one row (16-bit all-ones / all-zeros per pixel).
struct DirRow {
    uint32_t h0, h1, v0, v1, dm0, dm1;
};

__device__ __forceinline__ MRow msel(bool p, const MRow& a, const MRow& b) {
    MRow r;
    r.c0 = p ? a.c0 : b.c0; r.c1 = p ? a.c1 : b.c1;
    r.sm1 = p ? a.sm1 : b.sm1; r.s1 = p ? a.s1 : b.s1; r.s3 = p ? a.s3 : b.s3;
    return r;
}

__device__ __forceinline__ DirRow direction_masks(i16x2 gx0, i16x2 gx1, i16x2 gy0, i16x2 gy1,
                                                  i16x2 ax0, i16x2 ax1, i16x2 ay0, i16x2 ay1) {
    const i16x2 kH = {408, -169}, kV = {-169, 408};
    const uint32_t q00 = perm(W32(ax0), W32(ay0), 0x05040100u);  // (|Gy|, |Gx|) of x
    const uint32_t q01 = perm(W32(ax0), W32(ay0), 0x07060302u);  // (|Gy|, |Gx|) of x+1
    const uint32_t q10 = perm(W32(ax1), W32(ay1), 0x05040100u);
    const uint32_t q11 = perm(W32(ax1), W32(ay1), 0x07060302u);
    const int h00 = __builtin_amdgcn_sdot2(S(q00), kH, 0, false);
    const int h01 = __builtin_amdgcn_sdot2(S(q01), kH, 0, false);
    const int h10 = __builtin_amdgcn_sdot2(S(q10), kH, 0, false);
    const int h11 = __builtin_amdgcn_sdot2(S(q11), kH, 0, false);
    const int v00 = __builtin_amdgcn_sdot2(S(q00), kV, 0, false);
    const int v01 = __builtin_amdgcn_sdot2(S(q01), kV, 0, false);
    const int v10 = __builtin_amdgcn_sdot2(S(q10), kV, 0, false);
    const int v11 = __builtin_amdgcn_sdot2(S(q11), kV, 0, false);
    DirRow d;
    // sign of each dot product -> a 16-bit mask (low half from the first pixel)
    d.h0 = perm((uint32_t)h01, (uint32_t)h00, 0x0B0B0909u);
    d.h1 = perm((uint32_t)h11, (uint32_t)h10, 0x0B0B0909u);
    d.v0 = perm((uint32_t)v01, (uint32_t)v00, 0x0B0B0909u);
    d.v1 = perm((uint32_t)v11, (uint32_t)v10, 0x0B0B0909u);
    // anti-diagonal iff Gx and Gy have opposite signs
    d.dm0 = perm(0u, W32(gx0 ^ gy0), 0x09090808u);
    d.dm1 = perm(0u, W32(gx1 ^ gy1), 0x09090808u);
    return d;
}

// Suppression + thresholds for one lane's 4 pixels -> packed 2-bit byte.
__device__ __forceinline__ uint32_t classify4(const MRow& Mu, const MRow& Mc, const MRow& Md,
                                              const DirRow& dr, uint32_t low2, uint32_t high2,
                                              uint32_t vmask0, uint32_t vmask1) {
    uint32_t code[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const uint32_t mc = j ? Mc.c1 : Mc.c0;
        const uint32_t c_xm1 = j ? Mc.s1 : Mc.sm1, c_xp1 = j ? Mc.s3 : Mc.s1;
        const uint32_t u_c = j ? Mu.c1 : Mu.c0;
        const uint32_t u_xm1 = j ? Mu.s1 : Mu.sm1, u_xp1 = j ? Mu.s3 : Mu.s1;
        const uint32_t d_c = j ? Md.c1 : Md.c0;
        const uint32_t d_xm1 = j ? Md.s1 : Md.sm1, d_xp1 = j ? Md.s3 : Md.s1;
        const uint32_t mh = j ? dr.h1 : dr.h0, mv = j ? dr.v1 : dr.v0, mdm = j ? dr.dm1 : dr.dm0;
        // neighbour behind (p - d) and ahead (p + d) along the direction
        const uint32_t back = bsel(mh, c_xm1, bsel(mv, u_c, bsel(mdm, u_xp1, u_xm1)));
        const uint32_t fwd = bsel(mh, c_xp1, bsel(mv, d_c, bsel(mdm, d_xm1, d_xp1)));
        const uint32_t gt_back = W32(S(back) - S(mc));  // sign set iff M > back
        const uint32_t lt_fwd = W32(S(mc) - S(fwd));    // sign set iff M < fwd
        const uint32_t keep = gt_back & ~lt_fwd;
        const uint32_t strong = keep & W32(S(high2) - S(mc));  // M > high
        const uint32_t cand = keep & ~W32(S(mc) - S(low2));    // M >= low
        const u16x2 sh = {15, 15};
        code[j] = W32((U(cand) >> sh) + (U(strong) >> sh)) & (j ? vmask1 : vmask0);
    }
    const uint32_t z = code[0] | (code[1] << 4);
    return (z | (z >> 14)) & 0xFFu;
}

// The strip walk.  BORDER = false: every row and column the wave touches is
// inside the image and the input is 4-byte aligned, so no clamping or
// re-extension is needed.  BORDER = true: clamped loads and per-stage
// replication of the edge row / column.
template <int R, bool BORDER>
__device__ __forceinline__ void walk(const U8FwdArgs& a, int X0, int Y0, int lane) {
    const int H = a.H, W = a.W;
    const int c0 = X0 - 4 + 4 * lane;

    Border bd;
    uint32_t vmask0 = 0xFFFFFFFFu, vmask1 = 0xFFFFFFFFu;
    if (BORDER) {
        bd.left = X0 == 0;
        bd.right = X0 + kU8StripCols + 4 > W;
        bd.l0_lane = 1;
        const int off = W - 1 - (X0 - 4);  // position of column W-1 in the strip
        bd.lw_lane = min(off >> 2, kWave - 1);
        bd.lw_pair = (off >> 1) & 1;
        bd.lw_shift = (off & 1) * 16;
        bd.mL0 = (c0 < 0 ? 0xFFFFu : 0u) | (c0 + 1 < 0 ? 0xFFFF0000u : 0u);
        bd.mL1 = (c0 + 2 < 0 ? 0xFFFFu : 0u) | (c0 + 3 < 0 ? 0xFFFF0000u : 0u);
        bd.mR0 = (c0 >= W ? 0xFFFFu : 0u) | (c0 + 1 >= W ? 0xFFFF0000u : 0u);
        bd.mR1 = (c0 + 2 >= W ? 0xFFFFu : 0u) | (c0 + 3 >= W ? 0xFFFF0000u : 0u);
        vmask0 = ~bd.mR0;  // output columns inside the image
        vmask1 = ~bd.mR1;
    }
    const uint32_t low2 = ((uint32_t)a.low & 0xFFFFu) * 0x10001u;
    const uint32_t high2 = ((uint32_t)a.high & 0xFFFFu) * 0x10001u;
    const bool store_lane = lane >= 1 && lane <= 62 && (!BORDER || c0 < W);
    // Class bytes go out through an unconditional buffer store: lanes that do
    // not store carry an offset past the descriptor's range and the hardware
    // drops their writes.  A store behind a branch leaves the number of
    // outstanding memory operations unknown to the compiler, which then waits
    // for all of them -- the prefetched input rows included.
    const uint32_t soff = store_lane ? (uint32_t)(c0 >> 2) : 0x80000000u;

    // input rows are loaded kPF rows ahead of their use (a rolling queue);
    // border waves hold four byte loads per row, so they look fewer rows ahead
    constexpr int kPF = BORDER ? 6 : 12;
    auto load_row = [&](int i) -> uint32_t {
        if (BORDER) {
            const int y = min(max(Y0 - 4 + i, 0), H - 1);
            return load_px4_clamped(a.in + (int64_t)y * a.pitch, c0, W);
        }
        // buffer load: the row's base in scalar registers, the lane's offset
        // in one vector register (c0 >= 0 for interior waves)
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<uint8_t*>(a.in + (int64_t)(Y0 - 4 + i) * a.pitch), (short)0, 0x7fffffff, 0x00020000);
        return __builtin_amdgcn_raw_buffer_load_b32(rs, c0, 0, 0);
    };
    uint32_t q[kPF];
#pragma unroll
    for (int i = 0; i < kPF; ++i) q[i] = i < R + 8 ? load_row(i) : 0u;

    uint32_t hw0[5], hw1[5];                      // h rows vi-4 .. vi
    uint32_t dxw0[3], dxw1[3], sxw0[3], sxw1[3];  // rows b-2 .. b
    MRow mu, mc, md;                              // rows g-2, g-1, g
    DirRow dir_prev, dir_cur;                     // rows g-1, g

#pragma unroll
    for (int i = 0; i < R + 8; ++i) {
        // ---- Step 1a: horizontal blur of input row vi = Y0 - 4 + i
#pragma unroll
        for (int k = 0; k < 4; ++k) { hw0[k] = hw0[k + 1]; hw1[k] = hw1[k + 1]; }
        const uint32_t cur = q[0];
#pragma unroll
        for (int k = 0; k < kPF - 1; ++k) q[k] = q[k + 1];
        q[kPF - 1] = i + kPF < R + 8 ? load_row(i + kPF) : 0u;
        hblur(cur, hw0[4], hw1[4]);
        if (i < 4) continue;

        // ---- Step 1b: vertical blur, B row b = vi - 2
        const int b = Y0 - 6 + i;
        const u16x2 four = {4, 4}, six = {6, 6}, rnd = {128, 128}, eight = {8, 8};
        uint32_t B0 = W32(((U(hw0[0]) + U(hw0[4])) + (U(hw0[1]) + U(hw0[3])) * four +
                           U(hw0[2]) * six + rnd) >> eight);
        uint32_t B1 = W32(((U(hw1[0]) + U(hw1[4])) + (U(hw1[1]) + U(hw1[3])) * four +
                           U(hw1[2]) * six + rnd) >> eight);
        if (BORDER) fix_cols(B0, B1, bd);
        // Sobel row terms
        const uint32_t bl = from_left(B1), br = from_right(B0);
        const uint32_t Sm1 = align16(B0, bl), S1 = align16(B1, B0), S3 = align16(br, B1);
        const u16x2 two = {2, 2};
        uint32_t dx0 = W32(S(S1) - S(Sm1)), dx1 = W32(S(S3) - S(S1));
        uint32_t sx0 = W32(U(Sm1) + U(S1) + U(B0) * two), sx1 = W32(U(S1) + U(S3) + U(B1) * two);
        dxw0[0] = dxw0[1]; dxw0[1] = dxw0[2];
        dxw1[0] = dxw1[1]; dxw1[1] = dxw1[2];
        sxw0[0] = sxw0[1]; sxw0[1] = sxw0[2];
        sxw1[0] = sxw1[1]; sxw1[1] = sxw1[2];
        if (BORDER && b >= H) {  // rows below the image replicate row H-1
            dx0 = dxw0[1]; dx1 = dxw1[1]; sx0 = sxw0[1]; sx1 = sxw1[1];
        }
        dxw0[2] = dx0; dxw1[2] = dx1; sxw0[2] = sx0; sxw1[2] = sx1;
        if (BORDER && b == 0) {  // rows above the image replicate row 0
            dxw0[0] = dxw0[1] = dx0; dxw1[0] = dxw1[1] = dx1;
            sxw0[0] = sxw0[1] = sx0; sxw1[0] = sxw1[1] = sx1;
        }
        if (i < 6) continue;

        // ---- Step 2: gradients, strength and direction of row g = b - 1
        const int g = b - 1;
        const i16x2 gx0 = S(dxw0[0]) + S(dxw0[1]) * (i16x2){2, 2} + S(dxw0[2]);
        const i16x2 gx1 = S(dxw1[0]) + S(dxw1[1]) * (i16x2){2, 2} + S(dxw1[2]);
        const i16x2 gy0 = S(sxw0[2]) - S(sxw0[0]);
        const i16x2 gy1 = S(sxw1[2]) - S(sxw1[0]);
        const i16x2 ax0 = __builtin_elementwise_max(gx0, -gx0);
        const i16x2 ax1 = __builtin_elementwise_max(gx1, -gx1);
        const i16x2 ay0 = __builtin_elementwise_max(gy0, -gy0);
        const i16x2 ay1 = __builtin_elementwise_max(gy1, -gy1);
        uint32_t M0 = W32(U(W32(ax0)) + U(W32(ay0)));
        uint32_t M1 = W32(U(W32(ax1)) + U(W32(ay1)));
        dir_prev = dir_cur;
        dir_cur = direction_masks(gx0, gx1, gy0, gy1, ax0, ax1, ay0, ay1);

        if (BORDER) fix_cols(M0, M1, bd);
        MRow m;
        m.c0 = M0;
        m.c1 = M1;
        {
            const uint32_t ml = from_left(M1), mr = from_right(M0);
            m.sm1 = align16(M0, ml);
            m.s1 = align16(M1, M0);
            m.s3 = align16(mr, M1);
        }
        mu = mc;
        mc = md;
        if (BORDER) {
            md = msel(g >= H, mc, m);  // rows below the image replicate row H-1
            if (g == 0) { mu = m; mc = m; }  // rows above replicate row 0
        } else {
            md = m;
        }
        if (i < 8) continue;

        // ---- Step 3 + thresholds: row n = g - 1 (rows past the image store nothing)
        const int n = g - 1;
        const uint32_t byte = classify4(mu, mc, md, dir_prev, low2, high2, vmask0, vmask1);
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            a.cls + (int64_t)min(n, H - 1) * a.cpitch, (short)0, 0x7fffffff, 0x00020000);
        __builtin_amdgcn_raw_buffer_store_b8((uint8_t)byte, rs, (int)(BORDER && n >= H ? 0x80000000u : soff), 0, 0);
    }
}

template <int R>
__global__ void __launch_bounds__(kWGThreads)
k_u8_forward(U8FwdArgs a, int strips_x, int nwaves, int fast_ok) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wave_in_wg = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wg = xcd_remap(blockIdx.x, gridDim.x);
    const int wave = wg * kWavesPerWG + wave_in_wg;
    if (wave >= nwaves) return;
    const int strip = wave % strips_x;
    const int blk = wave / strips_x;
    const int X0 = strip * kU8StripCols;
    const int Y0 = blk * R;
    const bool interior = fast_ok && X0 >= 4 && X0 + kU8StripCols + 4 <= a.W && Y0 >= 4 &&
                          Y0 + R + 4 <= a.H;
    if (interior) walk<R, false>(a, X0, Y0, lane);
    else walk<R, true>(a, X0, Y0, lane);
}

template <int RRI, int RRE>
__global__ void __launch_bounds__(kWGThreads)
k_u8_forward_bal(U8FwdArgs a, U8Plan p, int fast_ok) {
    static_assert(RRE >= 4, "the top border block must cover the interior blocks' upper halo");
    const int lane = threadIdx.x & (kWave - 1);
    const int wave_in_wg = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wg = xcd_remap(blockIdx.x, gridDim.x);
    const int wave = wg * kWavesPerWG + wave_in_wg;
    if (wave >= p.nwaves) return;
    int X0, Y0;
    bool interior = false;
    if (wave < p.edge_waves) {
        const int es = wave % p.n_es;
        X0 = (es == 0 ? 0 : p.sr + es - 1) * kU8StripCols;
        Y0 = (wave / p.n_es) * RRE;
    } else {
        const int w = wave - p.edge_waves;
        const int blk = w / p.n_is;
        X0 = (1 + w % p.n_is) * kU8StripCols;
        if (blk == 0) {
            Y0 = 0;
        } else if (blk <= p.k) {
            Y0 = RRE + (blk - 1) * RRI;
            interior = true;
        } else {
            Y0 = RRE + p.k * RRI + (blk - 1 - p.k) * RRE;
        }
    }
    if (interior) {
        if (!(fast_ok && X0 >= 4 && X0 + kU8StripCols + 4 <= a.W && Y0 >= 4 && Y0 + RRI + 4 <= a.H))
            return;  // unreachable for a plan from make_u8_plan
        walk<RRI, false>(a, X0, Y0, lane);
    } else {
        walk<RRE, true>(a, X0, Y0, lane);
    }
}

// Batch forward: one wave per (image, strip, row block) task over all
// images of the batch.
template <int R>
__global__ void __launch_bounds__(kWGThreads)
k_u8_forward_batch(const BatchImage* imgs, const BatchDev* hdr) {
    const int lane = threadIdx.x & (kWave - 1);
    const int n = hdr->n, total = hdr->total_fwd;
    char* ws = hdr->ws;
    // one wave per task (image, strip, row block); the image by binary search
    const int tk = blockIdx.x * kWavesPerWG + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (tk >= total) return;
    int lo = 0, hi = n - 1;  // last image whose first task is <= tk
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (imgs[mid].fwd_base <= tk) lo = mid;
        else hi = mid - 1;
    }
    {
        const BatchImage& im = imgs[lo];
        U8FwdArgs a;
        a.in = im.in;
        a.pitch = im.pitch;
        a.H = im.H;
        a.W = im.W;
        a.low = hdr->low;
        a.high = hdr->high;
        a.cls = reinterpret_cast<uint8_t*>(ws + im.cls_off);
        a.cpitch = im.cpitch;
        const int local = tk - im.fwd_base;
        const int blk = local / im.fwd_strips_x;
        const int X0 = (local - blk * im.fwd_strips_x) * kU8StripCols;
        const int Y0 = blk * R;
        const bool fast_ok = ((uintptr_t)a.in % 4 == 0) && (a.pitch % 4 == 0);
        const bool interior = fast_ok && X0 >= 4 && X0 + kU8StripCols + 4 <= a.W && Y0 >= 4 &&
                              Y0 + R + 4 <= a.H;
        if (interior) walk<R, false>(a, X0, Y0, lane);
        else walk<R, true>(a, X0, Y0, lane);
    }
}

}  // namespace

hipError_t launch_u8_forward_batch(const BatchImage* imgs, const BatchDev* hdr, int rows, int total_fwd,
                                   hipStream_t s) {
    const int nwg = max(ceil_div(total_fwd, kWavesPerWG), 1);
    switch (rows) {
        case 48: hipLaunchKernelGGL(k_u8_forward_batch<48>, dim3(nwg), dim3(kWGThreads), 0, s, imgs, hdr); break;
        case 64: hipLaunchKernelGGL(k_u8_forward_batch<64>, dim3(nwg), dim3(kWGThreads), 0, s, imgs, hdr); break;
        case 96: hipLaunchKernelGGL(k_u8_forward_batch<96>, dim3(nwg), dim3(kWGThreads), 0, s, imgs, hdr); break;
        case 128: hipLaunchKernelGGL(k_u8_forward_batch<128>, dim3(nwg), dim3(kWGThreads), 0, s, imgs, hdr); break;
        default: hipLaunchKernelGGL(k_u8_forward_batch<32>, dim3(nwg), dim3(kWGThreads), 0, s, imgs, hdr); break;
    }
    return hipGetLastError();
}

int u8_forward_supported_rows(int rows) {
    return rows == 32 || rows == 48 || rows == 64 || rows == 96 || rows == 128;
}

template <int R>
static hipError_t launch_r(const U8FwdArgs& a, hipStream_t s) {
    const int strips_x = ceil_div(a.W, kU8StripCols);
    const int nwaves = strips_x * ceil_div(a.H, R);
    const int nwg = ceil_div(nwaves, kWavesPerWG);
    const int fast_ok = ((uintptr_t)a.in % 4 == 0) && (a.pitch % 4 == 0);
    hipLaunchKernelGGL(k_u8_forward<R>, dim3(nwg), dim3(kWGThreads), 0, s, a, strips_x, nwaves,
                       fast_ok);
    return hipGetLastError();
}

constexpr int kU8RRI = 40, kU8RRE = 20;  // balanced block heights (interior, border)

// The balanced split (32-row blocks everywhere when it would give fewer than
// 1024 waves, one per SIMD); rows_per_wave > 0 asks for 32-row blocks
// everywhere.
hipError_t launch_u8_forward(const U8FwdArgs& a, int rows_per_wave, hipStream_t s) {
    if (rows_per_wave <= 0) {
        const int fast_ok = ((uintptr_t)a.in % 4 == 0) && (a.pitch % 4 == 0);
        const U8Plan p = make_u8_plan(a.H, a.W, fast_ok, kU8RRI, kU8RRE);
        if (p.nwaves < 1024 || !u8_plan_ok(p, a.H, a.W, fast_ok, kU8RRI, kU8RRE)) return launch_r<32>(a, s);
        hipLaunchKernelGGL((k_u8_forward_bal<kU8RRI, kU8RRE>), dim3(ceil_div(p.nwaves, kWavesPerWG)),
                           dim3(kWGThreads), 0, s, a, p, fast_ok);
        return hipGetLastError();
    }
    return launch_r<32>(a, s);
}

}  // namespace canny
