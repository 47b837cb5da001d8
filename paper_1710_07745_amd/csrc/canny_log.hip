// Laplacian zero-crossing detector for gfx950 on uint8 images: the
// comparator the paper's introduction sets Canny against, the Laplace
// operator f_xx + f_yy, applied after the integer path's Step 1.
//   B = 5x5 binomial (1,4,6,4,1) per axis, one rounding (B = (S + 128) >> 8)
//   L = B(x-1) + B(x+1) + B(y-1) + B(y+1) - 4 B        (5-point Laplacian)
//   edges: (a) between 4-neighbours p, q whose L have strictly opposite
//          signs and |L(p) - L(q)| >= t, on the one nearer the zero (smaller
//          |L|; the earlier pixel in raster order on a tie);
//          (b) at a pixel with L = 0 whose left and right, or upper and lower,
//          neighbours have strictly opposite signs with |difference| >= t.
// Replicate borders at every stage; pairs reaching outside the image never
// cross (L is re-extended by copying the edge column / row, which gives equal
// values across the border).
//
// Same work layout as the integer Canny forward: a wave owns a 248-column
// strip, lane l holds the four columns c0 = X0 - 4 + 4l .. c0 + 3 as one
// dword (halo: 2 blur + 1 Laplacian + 1 crossing = 4 columns, so lanes 0 and
// 63 carry it), and walks its strip top to bottom with every stage's rows in
// registers:
//   input row -> horizontal binomial (5-row window) -> vertical binomial +
//   rounding (B) and its horizontal second difference (3-row window) ->
//   L (3-row window) -> crossing masks -> 4 edge bytes per lane.
// All arithmetic is packed 16-bit: |L| <= 1020, |L(p)| + |L(q)| <= 2040.
#include "canny_internal.h"
#include "canny_u8_common.h"

namespace canny {
namespace {

__device__ __forceinline__ i16x2 ashr15(i16x2 v) { return v >> (i16x2){15, 15}; }

// sign masks (all ones in a half where the value is < 0 / > 0) and |v|
struct Sgn {
    i16x2 neg, pos, abs;
};
__device__ __forceinline__ Sgn sgn(i16x2 v) {
    const i16x2 nv = (i16x2){0, 0} - v;
    return {ashr15(v), ashr15(nv), __builtin_elementwise_max(v, nv)};
}

// strictly opposite signs, and |a - b| = |a| + |b| >= t (masks per half)
__device__ __forceinline__ i16x2 crosses(const Sgn& a, const Sgn& b, i16x2 t2) {
    const i16x2 opp = (a.neg & b.pos) | (a.pos & b.neg);
    return opp & ~ashr15(a.abs + b.abs - t2);
}

// Edge masks of two pixels c (x, x+1) with their neighbours on the left
// (x-1, x), right (x+1, x+2), above and below.
__device__ __forceinline__ uint32_t edge_mask(i16x2 c, i16x2 l, i16x2 r, i16x2 u, i16x2 d, i16x2 t2) {
    const Sgn sc = sgn(c), sl = sgn(l), sr = sgn(r), su = sgn(u), sd = sgn(d);
    // (a) the pair with a later neighbour marks c when |c| <= |q|, with an
    // earlier neighbour when |c| < |q|
    i16x2 m = crosses(sc, sr, t2) & ~ashr15(sr.abs - sc.abs);
    m |= crosses(sc, sd, t2) & ~ashr15(sd.abs - sc.abs);
    m |= crosses(sc, sl, t2) & ashr15(sc.abs - sl.abs);
    m |= crosses(sc, su, t2) & ashr15(sc.abs - su.abs);
    // (b) c = 0 between opposite neighbours
    const i16x2 zero = ~(sc.neg | sc.pos);
    m |= zero & (crosses(sl, sr, t2) | crosses(su, sd, t2));
    return W32(m);
}

template <int R, bool BORDER>
__device__ __forceinline__ void log_walk(const LogArgs& a, int X0, int Y0, int lane, bool fast_ok) {
    const int H = a.H, W = a.W;
    const int c0 = X0 - 4 + 4 * lane;

    Border bd;
    bool fast = true;
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
        fast = fast_ok && c0 >= 0 && c0 + 4 <= W;
    }
    const i16x2 t2 = {(short)a.t, (short)a.t};
    const bool store_lane = lane >= 1 && lane <= 62 && (!BORDER || c0 < W);
    const bool full4 = !BORDER || c0 + 4 <= W;  // all four columns inside the image

    constexpr int kPF = 12;  // input rows loaded ahead of use
    auto load_row = [&](int i) -> uint32_t {
        if (BORDER) {
            const int y = min(max(Y0 - 4 + i, 0), H - 1);
            return load_px4(a.in + (int64_t)y * a.pitch, c0, W, fast);
        }
        const uint8_t* rowp = uniform_ptr(a.in + (int64_t)(Y0 - 4 + i) * a.pitch);
        return *reinterpret_cast<const uint32_t*>(rowp + (uint32_t)c0);
    };
    uint32_t q[kPF];
#pragma unroll
    for (int i = 0; i < kPF; ++i) q[i] = i < R + 8 ? load_row(i) : 0u;

    uint32_t hw0[5], hw1[5];                      // horizontal blur, rows vi-4 .. vi
    uint32_t bw0[3], bw1[3], xw0[3], xw1[3];      // B and its x second difference, rows b-2 .. b
    uint32_t lw0[3], lw1[3];                      // L, rows g-2 .. g

#pragma unroll
    for (int i = 0; i < R + 8; ++i) {
        // ---- horizontal binomial of input row vi = Y0 - 4 + i
#pragma unroll
        for (int k = 0; k < 4; ++k) { hw0[k] = hw0[k + 1]; hw1[k] = hw1[k + 1]; }
        const uint32_t cur = q[0];
#pragma unroll
        for (int k = 0; k < kPF - 1; ++k) q[k] = q[k + 1];
        q[kPF - 1] = i + kPF < R + 8 ? load_row(i + kPF) : 0u;
        hblur(cur, hw0[4], hw1[4]);
        if (i < 4) continue;

        // ---- vertical binomial + rounding: B row b = vi - 2; its x second
        // difference B(x-1) + B(x+1) - 4 B(x) (the Laplacian's row part)
        const int b = Y0 - 6 + i;
        const u16x2 four = {4, 4}, six = {6, 6}, rnd = {128, 128}, eight = {8, 8};
        uint32_t B0 = W32(((U(hw0[0]) + U(hw0[4])) + (U(hw0[1]) + U(hw0[3])) * four +
                           U(hw0[2]) * six + rnd) >> eight);
        uint32_t B1 = W32(((U(hw1[0]) + U(hw1[4])) + (U(hw1[1]) + U(hw1[3])) * four +
                           U(hw1[2]) * six + rnd) >> eight);
        if (BORDER) fix_cols(B0, B1, bd);
        const uint32_t bl = from_left(B1), br = from_right(B0);
        const uint32_t Sm1 = align16(B0, bl), S1 = align16(B1, B0), S3 = align16(br, B1);
        const i16x2 f4 = {4, 4};
        uint32_t X0v = W32(S(Sm1) + S(S1) - S(B0) * f4);
        uint32_t X1v = W32(S(S1) + S(S3) - S(B1) * f4);
        bw0[0] = bw0[1]; bw0[1] = bw0[2];
        bw1[0] = bw1[1]; bw1[1] = bw1[2];
        xw0[0] = xw0[1]; xw0[1] = xw0[2];
        xw1[0] = xw1[1]; xw1[1] = xw1[2];
        if (BORDER && b >= H) {  // rows below the image replicate row H-1
            B0 = bw0[1]; B1 = bw1[1]; X0v = xw0[1]; X1v = xw1[1];
        }
        bw0[2] = B0; bw1[2] = B1; xw0[2] = X0v; xw1[2] = X1v;
        if (BORDER && b == 0) {  // rows above the image replicate row 0
            bw0[0] = bw0[1] = B0; bw1[0] = bw1[1] = B1;
            xw0[0] = xw0[1] = X0v; xw1[0] = xw1[1] = X1v;
        }
        if (i < 6) continue;

        // ---- Laplacian of row g = b - 1
        const int g = b - 1;
        uint32_t L0 = W32(S(xw0[1]) + S(bw0[0]) + S(bw0[2]));
        uint32_t L1 = W32(S(xw1[1]) + S(bw1[0]) + S(bw1[2]));
        if (BORDER) fix_cols(L0, L1, bd);  // equal values across the border: no crossing
        lw0[0] = lw0[1]; lw0[1] = lw0[2];
        lw1[0] = lw1[1]; lw1[1] = lw1[2];
        if (BORDER && g >= H) { L0 = lw0[1]; L1 = lw1[1]; }
        lw0[2] = L0; lw1[2] = L1;
        if (BORDER && g == 0) { lw0[0] = lw0[1] = L0; lw1[0] = lw1[1] = L1; }
        if (i < 8) continue;

        // ---- zero crossings of row n = g - 1
        const int n = g - 1;
        if (BORDER && n >= H) continue;
        const uint32_t c0v = lw0[1], c1v = lw1[1];
        const uint32_t cl = from_left(c1v), cr = from_right(c0v);
        const uint32_t Lm1 = align16(c0v, cl), Lp1 = align16(c1v, c0v), Lp3 = align16(cr, c1v);
        const uint32_t m0 = edge_mask(S(c0v), S(Lm1), S(Lp1), S(lw0[0]), S(lw0[2]), t2);
        const uint32_t m1 = edge_mask(S(c1v), S(Lp1), S(Lp3), S(lw1[0]), S(lw1[2]), t2);
        const uint32_t bytes = perm(m1, m0, 0x07050301u);  // 0xFF / 0x00 per pixel
        if (store_lane) {
            uint8_t* erow = a.edges + (int64_t)n * a.epitch;
            if (full4 && a.estore4) {
                *reinterpret_cast<uint32_t*>(erow + c0) = bytes;
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (!BORDER || c0 + k < W) erow[c0 + k] = (uint8_t)(bytes >> (8 * k));
            }
            if (a.lap) {
                int16_t* lrow = a.lap + (int64_t)n * a.lpitch;
                const uint32_t lv[2] = {c0v, c1v};
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (!BORDER || c0 + k < W) lrow[c0 + k] = (int16_t)(lv[k >> 1] >> (16 * (k & 1)));
            }
        }
    }
}

constexpr int kLogRows = 32;  // output rows per wave

template <int R>
__global__ void __launch_bounds__(kWGThreads)
k_log_u8(LogArgs a, int strips_x, int nwaves, int fast_ok) {
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
    if (interior) log_walk<R, false>(a, X0, Y0, lane, true);
    else log_walk<R, true>(a, X0, Y0, lane, fast_ok);
}

}  // namespace

hipError_t launch_log_u8(const LogArgs& a, hipStream_t s) {
    const int strips_x = ceil_div(a.W, kU8StripCols);
    const int nwaves = strips_x * ceil_div(a.H, kLogRows);
    const int nwg = ceil_div(nwaves, kWavesPerWG);
    const int fast_ok = ((uintptr_t)a.in % 4 == 0) && (a.pitch % 4 == 0);
    hipLaunchKernelGGL(k_log_u8<kLogRows>, dim3(nwg), dim3(kWGThreads), 0, s, a, strips_x, nwaves,
                       fast_ok);
    return hipGetLastError();
}

}  // namespace canny
