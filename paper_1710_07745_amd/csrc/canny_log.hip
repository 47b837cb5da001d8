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
// Each pair of 4-neighbours is tested once (horizontal pairs within the row,
// the vertical pair with the row below, whose mark for the lower pixel is
// carried to the next row), which costs about half of testing all four
// neighbours from every pixel.
// All arithmetic is packed 16-bit: |L| <= 1020, |L(p)| + |L(q)| <= 2040.
#include "canny_internal.h"
#include "canny_u8_common.h"

namespace canny {
namespace {

// The crossing logic carries every decision in bit 15 of each 16-bit half
// (the sign bit of a packed value); the other bits are don't-cares.  So a
// negative test is the value itself, a positive test is its negation, and
// "a < b" is a - b: no shifts, no compares, no selects.  (Spelled as masks,
// x >> 15 & y, the compiler turned every test into per-element compares and
// selects.)  Only the final conversion to 0xFF / 0x00 per pixel shifts.
struct Sgn {
    i16x2 v, p, a;  // v: bit 15 iff < 0; p = -v: bit 15 iff > 0; a = |v|
};
__device__ __forceinline__ Sgn sgn(i16x2 v) {
    const i16x2 nv = (i16x2){0, 0} - v;
    return {v, nv, __builtin_elementwise_max(v, nv)};
}

// bit 15: strictly opposite signs, and |a - b| = |a| + |b| >= t
__device__ __forceinline__ i16x2 crosses(const Sgn& a, const Sgn& b, i16x2 t2) {
    const i16x2 opp = (a.v & b.p) | (a.p & b.v);
    return opp & ~(a.a + b.a - t2);
}

// bit 15 of each half -> 0xFFFF / 0x0000.  op_sel_hi:[0,1]: the high half's
// shift amount is the constant's low half too (by default it would read the
// constant's high 16 bits, 0, and leave the high half unshifted).
__device__ __forceinline__ uint32_t full_mask(uint32_t m) {
    uint32_t r;
    __asm__("v_pk_ashrrev_i16 %0, 15, %1 op_sel_hi:[0,1]" : "=v"(r) : "v"(m));
    return r;
}

// a lane's two packed registers (x, x+1), (x+2, x+3) moved one pixel: to the
// right neighbours (x+1, x+2), (x+3, x+4), or to the left ones (x-1, x)
__device__ __forceinline__ void to_right(uint32_t v0, uint32_t v1, uint32_t& r0, uint32_t& r1) {
    r0 = align16(v1, v0);
    r1 = align16(from_right(v0), v1);
}
__device__ __forceinline__ uint32_t to_left0(uint32_t v0, uint32_t v1) {
    return align16(v0, from_left(v1));
}

// E4: the edge rows take one 4-byte store per lane (4-byte aligned rows);
// else one byte store per pixel.  LAP: the Laplacian is written too.
template <int R, bool BORDER, bool E4, bool LAP>
__device__ __forceinline__ void log_walk(const LogArgs& a, int X0, int Y0, int lane) {
    static_assert(!(BORDER && E4), "border waves store bytes");
    const int H = a.H, W = a.W;
    const int c0 = X0 - 4 + 4 * lane;

    Border bd;
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
    }
    const i16x2 t2 = {(short)a.t, (short)a.t};
    const bool store_lane = lane >= 1 && lane <= 62 && (!BORDER || c0 < W);
    // Every store is issued unconditionally through a buffer descriptor; a
    // lane or pixel that must not be written carries an offset past the
    // range, and the hardware drops it.  With no store behind a branch the
    // compiler knows how many memory operations are outstanding and waits
    // only for the input row it needs, not for the prefetched ones.
    constexpr uint32_t kDrop = 0x80000000u;
    uint32_t boff[4], loff[4];  // byte offsets of the pixel in the edge and Laplacian rows
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const bool ok = store_lane && (!BORDER || c0 + k < W);
        boff[k] = ok ? (uint32_t)(c0 + k) : kDrop;
        loff[k] = ok ? 2u * (uint32_t)(c0 + k) : kDrop;
    }

    // input rows are loaded kPF rows ahead of their use; border waves hold
    // four byte loads per row, so they look fewer rows ahead
    constexpr int kPF = BORDER ? 6 : 12;
    auto load_row = [&](int i) -> uint32_t {
        if (BORDER) {
            const int y = min(max(Y0 - 4 + i, 0), H - 1);
            return load_px4_clamped(a.in + (int64_t)y * a.pitch, c0, W);
        }
        // the row's base in scalar registers, the lane's offset (c0 >= 0 for
        // interior waves) in one vector register
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<uint8_t*>(a.in + (int64_t)(Y0 - 4 + i) * a.pitch), (short)0, 0x7fffffff, 0x00020000);
        return __builtin_amdgcn_raw_buffer_load_b32(rs, c0, 0, 0);
    };
    uint32_t q[kPF];
#pragma unroll
    for (int i = 0; i < kPF; ++i) q[i] = i < R + 8 ? load_row(i) : 0u;

    uint32_t hw0[5], hw1[5];                      // horizontal blur, rows vi-4 .. vi
    uint32_t bw0[3], bw1[3], xw0[3], xw1[3];      // B and its x second difference, rows b-2 .. b
    uint32_t lw0[3], lw1[3];                      // L, rows g-2 .. g
    uint32_t down0 = 0, down1 = 0;                // marks of row n from the pair (n-1, n)

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

        // ---- zero crossings of row n = g - 1.  Each pair of 4-neighbours is
        // tested once, and its mark goes to the pixel nearer the zero (the
        // earlier one on a tie): horizontal pairs (x, x+1) of this row, the
        // vertical pair (n, n+1); the mark of (n-1, n) for row n comes from
        // the previous row's test (or, for the wave's first row, is tested
        // here).  Then the zeros between opposite neighbours.
        const int n = g - 1;  // rows past the image (border waves) store nothing
        const bool live = !BORDER || n < H;
        const Sgn c0s = sgn(S(lw0[1])), c1s = sgn(S(lw1[1]));
        const Sgn u0s = sgn(S(lw0[0])), u1s = sgn(S(lw1[0]));
        const Sgn d0s = sgn(S(lw0[2])), d1s = sgn(S(lw1[2]));
        // right neighbours (x+1, x+2), (x+3, x+4) and left ones (x-1, x)
        uint32_t rn0, rn1, rp0, rp1, ra0, ra1;
        to_right(W32(c0s.v), W32(c1s.v), rn0, rn1);
        to_right(W32(c0s.p), W32(c1s.p), rp0, rp1);
        to_right(W32(c0s.a), W32(c1s.a), ra0, ra1);
        const Sgn r0s = {S(rn0), S(rp0), S(ra0)}, r1s = {S(rn1), S(rp1), S(ra1)};
        const Sgn l0s = {S(to_left0(W32(c0s.v), W32(c1s.v))), S(to_left0(W32(c0s.p), W32(c1s.p))),
                         S(to_left0(W32(c0s.a), W32(c1s.a)))};
        // horizontal pairs starting at each pixel; the right pixel wins when
        // its |L| is strictly smaller (bit 15 of r.a - c.a)
        const i16x2 h0 = crosses(c0s, r0s, t2), h1 = crosses(c1s, r1s, t2);
        const i16x2 rw0 = r0s.a - c0s.a, rw1 = r1s.a - c1s.a;
        const uint32_t mR0 = W32(h0 & rw0), mR1 = W32(h1 & rw1);
        uint32_t m0 = W32(h0 & ~rw0) | align16(mR0, from_left(mR1));
        uint32_t m1 = W32(h1 & ~rw1) | align16(mR1, mR0);
        // vertical pair (n, n+1): the lower pixel wins when strictly smaller
        const i16x2 v0 = crosses(c0s, d0s, t2), v1 = crosses(c1s, d1s, t2);
        const i16x2 dw0 = d0s.a - c0s.a, dw1 = d1s.a - c1s.a;
        if (i == 8) {  // the wave's first row: the pair (n-1, n) has not been tested
            down0 = W32(crosses(u0s, c0s, t2) & (c0s.a - u0s.a));
            down1 = W32(crosses(u1s, c1s, t2) & (c1s.a - u1s.a));
        }
        m0 |= W32(v0 & ~dw0) | down0;
        m1 |= W32(v1 & ~dw1) | down1;
        down0 = W32(v0 & dw0);
        down1 = W32(v1 & dw1);
        // zeros (neither sign bit of v nor of -v set) between strictly
        // opposite left/right or upper/lower neighbours
        m0 |= W32(~(c0s.v | c0s.p) & (crosses(l0s, r0s, t2) | crosses(u0s, d0s, t2)));
        m1 |= W32(~(c1s.v | c1s.p) & (crosses(r0s, r1s, t2) | crosses(u1s, d1s, t2)));
        m0 = full_mask(m0);
        m1 = full_mask(m1);
        const uint32_t c0v = lw0[1], c1v = lw1[1];
        const uint32_t bytes = perm(m1, m0, 0x07050301u);  // 0xFF / 0x00 per pixel
        const int64_t nr = BORDER ? min(n, H - 1) : n;
        const __amdgpu_buffer_rsrc_t er = __builtin_amdgcn_make_buffer_rsrc(
            a.edges + nr * a.epitch, (short)0, 0x7fffffff, 0x00020000);
        if (E4) {
            __builtin_amdgcn_raw_buffer_store_b32(bytes, er, (int)(store_lane ? (uint32_t)c0 : kDrop), 0, 0);
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k)
                __builtin_amdgcn_raw_buffer_store_b8((uint8_t)(bytes >> (8 * k)), er, (int)(live ? boff[k] : kDrop), 0, 0);
        }
        if (LAP) {
            const __amdgpu_buffer_rsrc_t lr = __builtin_amdgcn_make_buffer_rsrc(
                a.lap + nr * a.lpitch, (short)0, 0x7fffffff, 0x00020000);
            const uint32_t lv[2] = {c0v, c1v};
#pragma unroll
            for (int k = 0; k < 4; ++k)
                __builtin_amdgcn_raw_buffer_store_b16((uint16_t)(lv[k >> 1] >> (16 * (k & 1))), lr,
                                                      (int)(live ? loff[k] : kDrop), 0, 0);
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
    if (a.lap) {
        if (interior && a.estore4) log_walk<R, false, true, true>(a, X0, Y0, lane);
        else if (interior) log_walk<R, false, false, true>(a, X0, Y0, lane);
        else log_walk<R, true, false, true>(a, X0, Y0, lane);
    } else {
        if (interior && a.estore4) log_walk<R, false, true, false>(a, X0, Y0, lane);
        else if (interior) log_walk<R, false, false, false>(a, X0, Y0, lane);
        else log_walk<R, true, false, false>(a, X0, Y0, lane);
    }
}

// Balanced launch (the integer forward's split, U8Plan): border blocks of
// RRE rows, interior blocks of RRI, so the border waves (clamped loads,
// per-stage replication) do not set the kernel's end.
template <int RRI, int RRE>
__global__ void __launch_bounds__(kWGThreads)
k_log_u8_bal(LogArgs a, U8Plan p, int fast_ok) {
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
        if (a.lap) {
            if (a.estore4) log_walk<RRI, false, true, true>(a, X0, Y0, lane);
            else log_walk<RRI, false, false, true>(a, X0, Y0, lane);
        } else {
            if (a.estore4) log_walk<RRI, false, true, false>(a, X0, Y0, lane);
            else log_walk<RRI, false, false, false>(a, X0, Y0, lane);
        }
    } else if (a.lap) {
        log_walk<RRE, true, false, true>(a, X0, Y0, lane);
    } else {
        log_walk<RRE, true, false, false>(a, X0, Y0, lane);
    }
}

constexpr int kLogRRI = 40, kLogRRE = 20;

}  // namespace

hipError_t launch_log_u8(const LogArgs& a, hipStream_t s) {
    const int fast_ok = ((uintptr_t)a.in % 4 == 0) && (a.pitch % 4 == 0);
    const U8Plan p = make_u8_plan(a.H, a.W, fast_ok, kLogRRI, kLogRRE);
    if (p.nwaves >= 1024 && u8_plan_ok(p, a.H, a.W, fast_ok, kLogRRI, kLogRRE)) {
        hipLaunchKernelGGL((k_log_u8_bal<kLogRRI, kLogRRE>), dim3(ceil_div(p.nwaves, kWavesPerWG)),
                           dim3(kWGThreads), 0, s, a, p, fast_ok);
        return hipGetLastError();
    }
    const int strips_x = ceil_div(a.W, kU8StripCols);
    const int nwaves = strips_x * ceil_div(a.H, kLogRows);
    const int nwg = ceil_div(nwaves, kWavesPerWG);
    hipLaunchKernelGGL(k_log_u8<kLogRows>, dim3(nwg), dim3(kWGThreads), 0, s, a, strips_x, nwaves,
                       fast_ok);
    return hipGetLastError();
}

}  // namespace canny
