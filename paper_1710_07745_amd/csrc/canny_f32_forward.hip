// Float Canny forward for gfx950: Steps 1-3 of the paper (Section 2.2.1) and
// the double threshold of Step 4 on fp32 images.
//
// Same work layout as the integer kernel: a wave owns a vertical strip, each
// lane holds 4 adjacent columns (one float4), the 64 lanes minus HL halo
// lanes on each side produce output, and the wave walks the strip top to
// bottom keeping every stage's rows in registers:
//   input rows (2R+1 window) -> vertical Gaussian V -> horizontal Gaussian B
//   (neighbour columns via DPP wave shifts) -> Sobel row terms dx, sx
//   (3-row window) -> Gx, Gy, M (3-row window) -> suppression + thresholds.
// Replicate borders per stage: input loads are clamped (which is exactly
// the clamp of the separable Gaussian, per axis); B and M are re-extended
// after they are formed (edge column / edge row copied outward).
//
// Relative thresholds need the image's largest strength before any pixel
// can be classified.  With absolute thresholds one launch classifies
// directly.  With relative thresholds (or when the largest strength is
// requested) the path is: a one-thread launch that clears the largest-strength
// word, the walk with a threshold-free epilogue that stores the strength with its sign
// carrying the suppression decision (+M kept, -M suppressed) and reduces the
// largest M into one word (atomicMax on the float bits, order-independent
// because the value is non-negative), then an elementwise pass that derives
// the thresholds from that word and writes the class map.  The walk, the
// expensive part, therefore runs once per image in both cases.  When only
// edges are asked for, the hysteresis pass classifies from the signed map
// itself; then each wave stores its largest M in a slot of its own and every
// hysteresis workgroup reduces the slots, so nothing has to clear a shared
// word before the walk (no extra launch).
//
// Accuracy: every stage before the strength is linear, so the walk filters
// X - off(x) instead of X, with off a line in the column, c + a x', taken
// from the wave's first input row (x' = column within the wave's window; a
// is 0 unless the row shows a trend across the strip).  The normalised
// symmetric Gaussian maps a line to itself (times the square of the taps'
// sum S), so the Sobel terms of the line are known exactly: nothing in y,
// and 8 S a in x, which is added back to Gx.  c and a lie on a power-of-two
// grid on which every off(x') is an exact fp32 value, so the subtraction is
// the only rounding the offset adds.  The fp32 accumulations then round at
// the magnitude of what the line does not explain (local contrast, not the
// image's level or a trend across the strip), and a constant image gives
// exactly zero.
//
// Suppression interpolates along the continuous gradient direction: with
// t = min(|Gx|,|Gy|) / max(|Gx|,|Gy|) and same = (Gx*Gy > 0),
//   dominant x: ahead = lerp(M(y,x+1), same ? M(y+1,x+1) : M(y-1,x+1), t)
//               behind = lerp(M(y,x-1), same ? M(y-1,x-1) : M(y+1,x-1), t)
//   dominant y: ahead = lerp(M(y+1,x), same ? M(y+1,x+1) : M(y+1,x-1), t)
//               behind = lerp(M(y-1,x), same ? M(y-1,x-1) : M(y-1,x+1), t)
// which is the 3x3-ring interpolation where the gradient line leaves the
// neighbourhood, written with the forward side fixed to the positive step of
// the dominant axis.
//
// SECTOR = true (one-launch mode only) is the variant with the direction
// quantised to the nearest multiple of 45 degrees, as in the integer path:
// suppression compares M with the two 8-neighbours p - d and p + d along it.
#include "../../include/canny.h"
#include "canny_internal.h"
#include "canny_f32_common.h"

namespace canny {
namespace {

struct MRowF {
    float c[4];
    float l, r;  // column c0-1 and c0+4
};

__device__ __forceinline__ MRowF selm(bool p, const MRowF& a, const MRowF& b) {
    MRowF r;
#pragma unroll
    for (int k = 0; k < 4; ++k) r.c[k] = p ? a.c[k] : b.c[k];
    r.l = p ? a.l : b.l;
    r.r = p ? a.r : b.r;
    return r;
}

template <int R>
struct WalkShape {
    static constexpr int HL = (R + 2 + 3) / 4;        // halo lanes per side
    static constexpr int SC = 4 * (kWave - 2 * HL);   // output columns per wave
    static constexpr int HR = R + 2;                  // halo rows per side
};

// One wave's strip: output rows Y0 .. Y0 + RR - 1, columns X0 .. X0 + SC - 1.
//
// The row loop is unrolled completely (every row index is a compile-time
// constant, so the per-row arrays below live in registers and sliding
// windows are plain renaming) and software-pipelined: iteration i blurs row
// i - R, forms the Sobel row terms of row i - R - 1, the gradients and
// strength of row i - R - 3 and the suppression of row i - R - 5 (row
// numbers relative to the first input row Y0 - HR).  Each stage reads only
// what earlier iterations produced, so the four stages of one iteration are
// independent instruction streams the scheduler can interleave, instead of
// one long dependency chain per row.
//
// EDGE = false is the interior case (every lane and every row inside the
// image, rows 16-byte aligned): no clamps and no replicate fix-ups.  EDGE =
// true handles strips and rows that touch the image border: clamped loads,
// edge columns copied outward, and the rows above row 0 / below row H-1
// replaced by the edge row where a stage reads them.
typedef float f32x4v __attribute__((ext_vector_type(4)));
typedef unsigned u32x4v __attribute__((ext_vector_type(4)));

// Work split of a balanced walk launch (large images).  Strips that touch the
// left or right border (or every strip when rows are not 16-byte aligned),
// and the top and bottom row blocks of the others, take the border variant,
// which costs about 1.5x the interior one per row; so border blocks are RRE
// rows tall and interior blocks RRI > RRE rows, which evens out the waves'
// durations (with one block height the border waves set the kernel's end).
//   waves [0, edge_waves): border strips {0} and [sr, strips_x), block-major;
//   the rest: interior strips [1, sr), block-major, per strip one top border
//   block [0, RRE), k interior blocks from row RRE, then nb border blocks.
struct WalkPlan {
    int nwaves, edge_waves;
    int n_es, sr, n_is;  // border strips, first right border strip, interior strips
    int k, nb;           // interior / bottom border blocks per interior strip
};

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    return v;  // a butterfly: every lane adds the same two operands per step
}

// The offset line off(x') = c + a x' of a wave, x' = 4 lane + k in 0..255,
// from the wave's first input row.  Two candidates: the constant midpoint of
// the row's range (a = 0), and a line with the least-squares slope and the
// midpoint of what it leaves.  The line is taken only where it at least
// halves the row's largest deviation from the offset: a trend across the
// strip.  A tilt fitted to ordinary content would help the first row and
// hurt the rows below it.  A line is rounded to the grid q = 2^(e - 21) with
// |c| + 255 |a| < 2^e; then |c|, |a x'| and |off| stay below 2^22 q, so
// fmaf(a, x', c) is exact.  Any line gives the same result in exact
// arithmetic (its Gaussian and Sobel terms are added back); the choice only
// keeps the filtered values small.
struct OffsetLine { float a, c; };

__device__ __forceinline__ OffsetLine offset_line(const F4& r0, int lane) {
    float sx = 0.0f;
#pragma unroll
    for (int k = 0; k < 4; ++k) sx = fmaf((float)(4 * lane + k) - 127.5f, r0.v[k], sx);
    const float lo = wave_min(fminf(fminf(r0.v[0], r0.v[1]), fminf(r0.v[2], r0.v[3])));
    const float hi = wave_max(fmaxf(fmaxf(r0.v[0], r0.v[1]), fmaxf(r0.v[2], r0.v[3])));
    sx = wave_sum(sx);
    const float a = sx * (1.0f / 1398080.0f);  // sum of (x' - 127.5)^2, x' = 0..255
    float rl = r0.v[0], rh = r0.v[0];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float e = fmaf(-a, (float)(4 * lane + k), r0.v[k]);
        rl = k ? fminf(rl, e) : e;
        rh = k ? fmaxf(rh, e) : e;
    }
    rl = wave_min(rl);
    rh = wave_max(rh);
    OffsetLine ol{0.0f, 0.5f * lo + 0.5f * hi};
    const float c = 0.5f * rl + 0.5f * rh;
    const float A = fabsf(c) + 255.0f * fabsf(a);
    if (rh - rl <= 0.5f * (hi - lo) && A > 1e-30f && A < 1e30f) {
        int e;
        (void)frexpf(A, &e);  // A < 2^e
        const float q = ldexpf(1.0f, e - 21), inv_q = ldexpf(1.0f, 21 - e);
        ol.a = rintf(a * inv_q) * q;
        ol.c = rintf(c * inv_q) * q;
    }
    ol.a = bc<float>(__builtin_amdgcn_readfirstlane(bc<int>(ol.a)));
    ol.c = bc<float>(__builtin_amdgcn_readfirstlane(bc<int>(ol.c)));
    return ol;
}

// Returns the wave's largest M as float bits (0 unless SIGNED), in every lane.
template <int R, int RR, bool SIGNED, bool SECTOR, bool EDGE>
__device__ __forceinline__ uint32_t f32_walk(const F32FwdArgs& a, int X0, int Y0, int lane, int fast_ok) {
    static_assert(!(SIGNED && SECTOR), "the four-sector variant classifies in the walk");
    constexpr int HL = WalkShape<R>::HL;
    constexpr int HR = WalkShape<R>::HR;
    constexpr int NI = RR + 2 * HR;          // input rows
    constexpr int PF = 4;                    // rows loaded ahead of use
    constexpr int TB0 = R, TB1 = RR + R + 3;      // rows blurred / Sobel terms
    constexpr int TG0 = R + 1, TG1 = RR + R + 2;  // rows with gradients and strength
    constexpr int TN0 = R + 2, TN1 = RR + R + 1;  // output rows
    constexpr int NIT = TN1 + R + 5 + 1;          // iterations (last: suppression of TN1)
    const int H = a.H, W = a.W;
    const int c0 = X0 - 4 * HL + 4 * lane;
    const int ybase = Y0 - HR;  // absolute row of relative row 0

    BorderF bd;
    bd.left = X0 == 0;
    bd.right = X0 + WalkShape<R>::SC + 4 * HL > W;
    bd.l0_lane = HL;
    {
        const int off = W - 1 - (X0 - 4 * HL);
        bd.lw_lane = min(off >> 2, kWave - 1);
        bd.lw_px = off & 3;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        bd.outL[k] = c0 + k < 0;
        bd.outR[k] = c0 + k >= W;
    }
    const bool out_lane = lane >= HL && lane < kWave - HL;
    const uint32_t soff = out_lane ? (uint32_t)c0 * 4u : 0x80000000u;

    float g[R + 1];
#pragma unroll
    for (int j = 0; j <= R; ++j) g[j] = a.g[j];

    // edge strips read every pixel with a clamped column index (4 loads per
    // row, no divergence); interior strips read one float4 per lane
    int cx[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) cx[k] = min(max(c0 + k, 0), W - 1);
    auto fetch = [&](int t) -> F4 {
        F4 r;
        if (EDGE) {
            const int y = min(max(ybase + t, 0), H - 1);
            const float* row = a.in + (int64_t)y * a.pitch;
#pragma unroll
            for (int k = 0; k < 4; ++k) r.v[k] = row[cx[k]];
        } else {
            const float4 q = *reinterpret_cast<const float4*>(a.in + (int64_t)(ybase + t) * a.pitch + c0);
            r.v[0] = q.x; r.v[1] = q.y; r.v[2] = q.z; r.v[3] = q.w;
        }
        return r;
    };
    F4 in[NI];
#pragma unroll
    for (int k = 0; k < PF && k < NI; ++k) in[k] = fetch(k);

    // offset plane subtracted from every input value (see the file comment)
    const OffsetLine ol = offset_line(in[0], lane);
    float off[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) off[k] = fmaf(ol.a, (float)(4 * lane + k), ol.c);  // exact
    // the blurred window is B - S (c + a x') with S the square of the taps'
    // exact sum, so every horizontal difference of it lacks 2 S a, and Gx
    // (1, 2, 1 of them) lacks 8 S a; in border strips the replicated columns
    // of B need S a (edge - x) on top of the copied edge value
    float gsum = g[0];
#pragma unroll
    for (int j = 1; j <= R; ++j) gsum = fmaf(2.0f, g[j], gsum);
    const float Sa = gsum * gsum * ol.a;
    const float gx_fix = 8.0f * Sa;
    float bfix[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        bfix[k] = bd.outL[k] ? Sa * (float)(-(c0 + k)) : (bd.outR[k] ? Sa * (float)(W - 1 - (c0 + k)) : 0.0f);

    // per-row values, indexed by relative row (compile-time indices only)
    F4 Bv[NI], dxv[NI], sxv[NI], gxv[NI], gyv[NI];
    MRowF mv[NI];
    float mmax = 0.0f;  // largest M of the rows this wave outputs

#pragma unroll
    for (int i = 0; i < NIT; ++i) {
        if (i + PF < NI) in[i + PF] = fetch(i + PF);
        if (i < NI) {
#pragma unroll
            for (int q = 0; q < 4; ++q) in[i].v[q] -= off[q];
        }

        // ---- Step 3 + thresholds: suppression of row tD
        const int tD = i - R - 5;
        if (tD >= TN0 && tD <= TN1) {
            const int n = ybase + tD;
            if (!EDGE || n < H) {
                const MRowF& c = mv[tD];
                MRowF u = mv[tD - 1], d = mv[tD + 1];
                if (EDGE) {  // rows -1 and H replicate rows 0 and H-1
                    u = selm(n == 0, c, u);
                    d = selm(n == H - 1, c, d);
                }
                uint32_t byte = 0;
                F4 sv;
                float rmax = 0.0f;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const float mc = c.c[k];
                    const float cl = k == 0 ? c.l : c.c[k - 1], cr = k == 3 ? c.r : c.c[k + 1];
                    const float ul = k == 0 ? u.l : u.c[k - 1], uc = u.c[k], ur = k == 3 ? u.r : u.c[k + 1];
                    const float dl = k == 0 ? d.l : d.c[k - 1], dc = d.c[k], dr = k == 3 ? d.r : d.c[k + 1];
                    const float gxk = gxv[tD].v[k], gyk = gyv[tD].v[k];
                    const float ax = fabsf(gxk), ay = fabsf(gyk);
                    const bool domx = ax >= ay;
                    const bool same = gxk * gyk > 0.0f;
                    const float mn = fminf(ax, ay), mxv = fmaxf(ax, ay);
                    const float fp = domx ? cr : dc;
                    const float fd = same ? dr : (domx ? ur : dl);
                    const float bp = domx ? cl : uc;
                    const float bdg = same ? ul : (domx ? dl : ur);
                    // with t = mn / mxv the interpolated neighbours are fp + t (fd - fp)
                    // and bp + t (bdg - bp); both sides are scaled by mxv > 0 instead
                    // of dividing (mxv = 0 implies mc = 0, which is never kept), as
                    // fd mn + fp (mxv - mn) with the difference shared by both sides
                    const float rest = mxv - mn;
                    const float ahead = fmaf(fd, mn, fp * rest);
                    const float behind = fmaf(bdg, mn, bp * rest);
                    const float ms = mc * mxv;
                    bool keep = mc > 0.0f && ms > behind && ms >= ahead;
                    if (SECTOR) {
                        // four-sector direction (nearest multiple of 45 degrees):
                        // axis x if ay < tan(22.5) ax, axis y if ay > tan(67.5) ax,
                        // else the diagonal (1, 1) (Gx, Gy of one sign) or (1, -1);
                        // compare with p - d (strictly) and p + d
                        const bool on_x = ay < 0.41421356f * ax, on_y = ay > 2.41421356f * ax;
                        float back = same ? ul : ur, fwd = same ? dr : dl;
                        back = on_y ? uc : back;
                        fwd = on_y ? dc : fwd;
                        back = on_x ? cl : back;
                        fwd = on_x ? cr : fwd;
                        keep = mc > 0.0f && mc > back && mc >= fwd;
                    }
                    if (SIGNED) {
                        // two selects on compare results instead of one on their
                        // conjunction (no scalar mask arithmetic between vector ops);
                        // M = 0 gives +-0, which reads as not kept (only > 0 is)
                        float t = ms >= ahead ? mc : -mc;
                        __asm__("" : "+v"(t));
                        sv.v[k] = ms > behind ? t : -mc;
                        if (!EDGE || !bd.outR[k]) rmax = fmaxf(rmax, mc);
                    } else {
                        const uint32_t code = (keep && mc > a.high) ? 2u : ((keep && mc >= a.low) ? 1u : 0u);
                        if (!EDGE || !bd.outR[k]) byte |= code << (2 * k);
                    }
                }
                if (SIGNED) {
                    // an opaque running max: otherwise the compiler may turn the chain
                    // of maxima into one reduction at the end and keep every row's M alive
                    mmax = fmaxf(mmax, rmax);
                    __asm__ volatile("" : "+v"(mmax));
                }
                if (SIGNED && !EDGE) {
                    // unconditional buffer store: halo lanes carry an offset past the
                    // descriptor's range, so the hardware drops their writes; no branch
                    // around the store keeps the load-wait counts exact
                    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                        a.smag + (int64_t)n * a.spitch, (short)0, 0x7fffffff, 0x00020000);
                    f32x4v q = {sv.v[0], sv.v[1], sv.v[2], sv.v[3]};
                    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4v, q), rs, (int)soff, 0, 0);
                } else if (out_lane && (!EDGE || c0 < W)) {
                    if (SIGNED) {
                        // row pitch is W rounded up to 4, so the quad store stays inside the row
                        *reinterpret_cast<float4*>(a.smag + (int64_t)n * a.spitch + c0) =
                            make_float4(sv.v[0], sv.v[1], sv.v[2], sv.v[3]);
                    } else {
                        a.cls[(int64_t)n * a.cpitch + (c0 >> 2)] = (uint8_t)byte;
                        if (a.mag) {
                            float* mrow = a.mag + (int64_t)n * W;
#pragma unroll
                            for (int k = 0; k < 4; ++k)
                                if (!EDGE || !bd.outR[k]) mrow[c0 + k] = c.c[k];
                        }
                    }
                }
            }
        }

        // ---- Step 2b: gradients and strength of row tC
        const int tC = i - R - 3;
        if (tC >= TG0 && tC <= TG1) {
            F4 dm = dxv[tC - 1], dp = dxv[tC + 1], sm = sxv[tC - 1], sp = sxv[tC + 1];
            if (EDGE) {  // rows -1 and H replicate rows 0 and H-1
                const int y = ybase + tC;
                dm = sel4(y == 0, dxv[tC], dm);
                sm = sel4(y == 0, sxv[tC], sm);
                dp = sel4(y == H - 1, dxv[tC], dp);
                sp = sel4(y == H - 1, sxv[tC], sp);
            }
            F4 M;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const float gx = fmaf(2.0f, dxv[tC].v[k], dm.v[k] + dp.v[k]) + gx_fix;
                const float gy = sp.v[k] - sm.v[k];
                gxv[tC].v[k] = gx;
                gyv[tC].v[k] = gy;
                // hardware square root: within an ulp, far inside the 1e-5 tolerance
                M.v[k] = __builtin_amdgcn_sqrtf(fmaf(gx, gx, gy * gy));
            }
            if (EDGE) fix_cols(M, bd);
#pragma unroll
            for (int k = 0; k < 4; ++k) mv[tC].c[k] = M.v[k];
            mv[tC].l = from_left_f(M.v[3]);
            mv[tC].r = from_right_f(M.v[0]);
        }

        // ---- Step 2a: Sobel row terms of row tB
        const int tB = i - R - 1;
        if (tB >= TB0 && tB <= TB1) {
            const F4& B = Bv[tB];
            const float bl = from_left_f(B.v[3]), br = from_right_f(B.v[0]);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const float xm = k == 0 ? bl : B.v[k - 1];
                const float xp = k == 3 ? br : B.v[k + 1];
                dxv[tB].v[k] = xp - xm;
                sxv[tB].v[k] = fmaf(2.0f, B.v[k], xm + xp);
            }
        }

        // ---- Step 1: Gaussian of row tA (vertical taps, then horizontal)
        const int tA = i - R;
        if (tA >= TB0 && tA <= TB1) {
            F4 V;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                float acc = g[0] * in[tA].v[k];
#pragma unroll
                for (int j = 1; j <= R; ++j) acc = fmaf(g[j], in[tA - j].v[k] + in[tA + j].v[k], acc);
                V.v[k] = acc;
            }
            float ext[4 + 2 * R];
#pragma unroll
            for (int e = -R; e < 4 + R; ++e) ext[e + R] = lane_ext(V, e);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                float acc = g[0] * ext[k + R];
#pragma unroll
                for (int j = 1; j <= R; ++j) acc = fmaf(g[j], ext[k + R - j] + ext[k + R + j], acc);
                Bv[tA].v[k] = acc;
            }
            if (EDGE) {
                fix_cols(Bv[tA], bd);
#pragma unroll
                for (int k = 0; k < 4; ++k) Bv[tA].v[k] += bfix[k];
            }
        }
    }

    return SIGNED ? bc<uint32_t>(wave_max(out_lane ? mmax : 0.0f)) : 0u;
}

// A wave's largest M: into its own slot when the consumer reduces the slots
// (every wave of the launch stores one, zeros included), else into the
// shared word (atomicMax on non-negative float bits, order-independent).
template <bool SIGNED>
__device__ __forceinline__ void publish_max(const F32FwdArgs& a, int wave, int lane, uint32_t v) {
    if (!SIGNED) return;
    if (a.maxslots) {
        if (lane == 0) a.maxslots[wave] = v;
    } else if (lane == 0 && v) {
        atomicMax(a.maxbits, v);
    }
}

// At least 3 waves per SIMD (<= 168 VGPRs); radii >= 6 need a longer input
// window and are allowed 2 (<= 256 VGPRs) rather than spill.
template <int R, int RR, bool SIGNED, bool SECTOR>
__global__ void __launch_bounds__(kWGThreads) __attribute__((amdgpu_waves_per_eu(R >= 6 ? 2 : 3)))
k_f32_forward(F32FwdArgs a, int strips_x, int nwaves, int fast_ok) {
    constexpr int HL = WalkShape<R>::HL;
    constexpr int SC = WalkShape<R>::SC;
    constexpr int HR = WalkShape<R>::HR;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave_in_wg = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wg = xcd_remap(blockIdx.x, gridDim.x);
    const int wave = wg * kWavesPerWG + wave_in_wg;
    if (wave >= nwaves) return;
    const int strip = wave % strips_x;
    const int blk = wave / strips_x;
    const int X0 = strip * SC;
    const int Y0 = blk * RR;
    const bool interior = fast_ok && X0 - 4 * HL >= 0 && X0 + SC + 4 * HL <= a.W &&
                          Y0 - HR >= 0 && Y0 + RR + HR <= a.H;
    const uint32_t v = interior ? f32_walk<R, RR, SIGNED, SECTOR, false>(a, X0, Y0, lane, fast_ok)
                                : f32_walk<R, RR, SIGNED, SECTOR, true>(a, X0, Y0, lane, fast_ok);
    publish_max<SIGNED>(a, wave, lane, v);
}

// Balanced launch: interior blocks of RRI rows, border blocks of RRE rows
// (see WalkPlan).  The task decides the variant; the interior conditions hold
// by construction and are checked again before the unclamped walk.
template <int R, int RRI, int RRE, bool SIGNED, bool SECTOR>
__global__ void __launch_bounds__(kWGThreads) __attribute__((amdgpu_waves_per_eu(R >= 6 ? 2 : 3)))
k_f32_forward_bal(F32FwdArgs a, WalkPlan p, int fast_ok) {
    constexpr int HL = WalkShape<R>::HL;
    constexpr int SC = WalkShape<R>::SC;
    constexpr int HR = WalkShape<R>::HR;
    static_assert(RRE >= HR, "the top border block must cover the interior blocks' upper halo");
    const int lane = threadIdx.x & (kWave - 1);
    const int wave_in_wg = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wg = xcd_remap(blockIdx.x, gridDim.x);
    const int wave = wg * kWavesPerWG + wave_in_wg;
    if (wave >= p.nwaves) return;
    int X0, Y0;
    bool interior = false;
    if (wave < p.edge_waves) {
        const int es = wave % p.n_es;
        X0 = (es == 0 ? 0 : p.sr + es - 1) * SC;
        Y0 = (wave / p.n_es) * RRE;
    } else {
        const int w = wave - p.edge_waves;
        const int blk = w / p.n_is;
        X0 = (1 + w % p.n_is) * SC;
        if (blk == 0) {
            Y0 = 0;
        } else if (blk <= p.k) {
            Y0 = RRE + (blk - 1) * RRI;
            interior = true;
        } else {
            Y0 = RRE + p.k * RRI + (blk - 1 - p.k) * RRE;
        }
    }
    uint32_t v = 0;
    if (interior) {
        if (fast_ok && X0 - 4 * HL >= 0 && X0 + SC + 4 * HL <= a.W && Y0 - HR >= 0 &&
            Y0 + RRI + HR <= a.H)  // always true for a plan from make_walk_plan
            v = f32_walk<R, RRI, SIGNED, SECTOR, false>(a, X0, Y0, lane, fast_ok);
    } else {
        v = f32_walk<R, RRE, SIGNED, SECTOR, true>(a, X0, Y0, lane, fast_ok);
    }
    publish_max<SIGNED>(a, wave, lane, v);
}

constexpr int kRowThreads = 256;  // one workgroup walks whole rows
typedef float f32x4 __attribute__((ext_vector_type(4)));


constexpr int kRowBatch = 8;  // rows a thread reads per batch (loads in flight)

// Clears the largest-strength word the walk reduces into (atomicMax of
// non-negative float bits); a kernel rather than a memset, so the sequence
// can be recorded into a graph and replayed.
__global__ void __launch_bounds__(kWave) k_f32_clear_max(uint32_t* maxbits) {
    if (threadIdx.x == 0) *maxbits = 0u;
}

// Thresholds and classes from the signed strength map: a pixel is kept iff
// its stored value is positive (M > 0 and not suppressed); then strong iff
// M > high, weak iff M >= low, with low/high scaled by the largest M when
// thresholds are relative.  Workgroup b owns rows b, b + gridDim.x, ...; a
// thread takes quad columns q = threadIdx.x + 256 j (one class byte each,
// so a wave's loads and stores are contiguous), kRowBatch rows per batch.
__global__ void __launch_bounds__(kRowThreads)
k_f32_classify(F32FwdArgs a) {
    const float mx = bc<float>(a.maxbits[0]);
    const float lo = a.relative ? a.low * mx : a.low;
    const float hi = a.relative ? a.high * mx : a.high;
    if (a.max_out && blockIdx.x == 0 && threadIdx.x == 0) *a.max_out = mx;
    const int W = a.W;
    const int nq = (W + 3) >> 2;  // quads of the row (the pitch holds them all)
    const int nrows = (a.H - (int)blockIdx.x + (int)gridDim.x - 1) / (int)gridDim.x;
    const bool mag4 = a.mag && (W % 4 == 0) && ((uintptr_t)a.mag % 16 == 0);
    for (int q = threadIdx.x; q < nq; q += kRowThreads) {
        for (int k0 = 0; k0 < nrows; k0 += kRowBatch) {
            f32x4 v[kRowBatch];
#pragma unroll
            for (int u = 0; u < kRowBatch; ++u) {
                const int y = (int)blockIdx.x + (k0 + u) * (int)gridDim.x;
                if (k0 + u < nrows) v[u] = reinterpret_cast<const f32x4*>(a.smag + (int64_t)y * a.spitch)[q];
            }
#pragma unroll
            for (int u = 0; u < kRowBatch; ++u) {
                if (k0 + u >= nrows) break;
                const int y = (int)blockIdx.x + (k0 + u) * (int)gridDim.x;
                const float e[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
                uint32_t byte = 0;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const uint32_t code =
                        (4 * q + k < W && e[k] > 0.0f) ? (e[k] > hi ? 2u : (e[k] >= lo ? 1u : 0u)) : 0u;
                    byte |= code << (2 * k);
                }
                a.cls[(int64_t)y * a.cpitch + q] = (uint8_t)byte;
                if (a.mag) {
                    float* mrow = a.mag + (int64_t)y * W;
                    if (mag4) {
                        *reinterpret_cast<float4*>(mrow + 4 * q) =
                            make_float4(fabsf(e[0]), fabsf(e[1]), fabsf(e[2]), fabsf(e[3]));
                    } else {
#pragma unroll
                        for (int k = 0; k < 4; ++k)
                            if (4 * q + k < W) mrow[4 * q + k] = fabsf(e[k]);
                    }
                }
            }
        }
    }
}

// row-owning workgroups of the classify pass: few enough that each owns a
// full batch of rows on large images
int rows_grid(int H) { return min(H, 512); }

// One walk launch with RR output rows per wave.
template <int R, int RR, bool SIGNED, bool SECTOR>
void launch_walk(const F32FwdArgs& a, int fast_ok, hipStream_t s) {
    const int strips_x = ceil_div(a.W, WalkShape<R>::SC);
    const int nwaves = strips_x * ceil_div(a.H, RR);
    const int nwg = ceil_div(nwaves, kWavesPerWG);
    hipLaunchKernelGGL((k_f32_forward<R, RR, SIGNED, SECTOR>), dim3(nwg), dim3(kWGThreads), 0, s, a,
                       strips_x, nwaves, fast_ok);
}

constexpr int kRRI = 40, kRRE = 23;  // balanced block heights (interior, border)

template <int R>
WalkPlan make_walk_plan(int H, int W, int fast_ok) {
    constexpr int SC = WalkShape<R>::SC, HL = WalkShape<R>::HL;
    WalkPlan p{};
    const int strips_x = ceil_div(W, SC);
    int sr = strips_x;  // first strip whose right halo leaves the image
    if (!fast_ok) {
        sr = 1;
    } else {
        for (int s = 1; s < strips_x; ++s)
            if ((int64_t)(s + 1) * SC + 4 * HL > W) {
                sr = s;
                break;
            }
    }
    if (strips_x == 1) sr = 1;
    p.sr = sr;
    p.n_es = 1 + (strips_x - sr);
    p.n_is = sr - 1;
    p.k = H >= 2 * kRRE ? (H - 2 * kRRE) / kRRI : 0;
    p.nb = ceil_div(max(0, H - kRRE - p.k * kRRI), kRRE);
    p.edge_waves = p.n_es * ceil_div(H, kRRE);
    p.nwaves = p.edge_waves + p.n_is * (1 + p.k + p.nb);
    return p;
}

// The interior conditions the balanced kernel relies on, checked on the host
// (they hold by construction): every interior block and every interior strip
// has its halo inside the image, and interior waves read 16-byte aligned rows.
template <int R>
bool walk_plan_ok(const WalkPlan& p, int H, int W, int fast_ok) {
    constexpr int SC = WalkShape<R>::SC, HL = WalkShape<R>::HL, HR = WalkShape<R>::HR;
    if (p.n_is == 0 || p.k == 0) return true;  // no interior block
    return fast_ok && kRRE - HR >= 0 && kRRE + p.k * kRRI + HR <= H && SC - 4 * HL >= 0 &&
           (int64_t)p.sr * SC + 4 * HL <= W;  // last interior strip is sr - 1
}

// Rows per wave: a wave walks its strip serially, so long strips suit large
// images (halo rows amortised) and short ones small images (more waves in
// flight).  The balanced split unless that leaves fewer than 1024 waves (one
// per SIMD); then 8 rows per wave.
// interior waves may read rows as aligned 16-byte quads
int walk_fast_ok(const F32FwdArgs& a) { return ((uintptr_t)a.in % 16 == 0) && (a.pitch % 4 == 0); }

template <int R>
bool use_balanced(const WalkPlan& p, int H, int W, int fast_ok) {
    return p.nwaves >= 1024 && walk_plan_ok<R>(p, H, W, fast_ok);
}

template <int R>
int walk_waves_r(int H, int W, int fast_ok) {
    const WalkPlan p = make_walk_plan<R>(H, W, fast_ok);
    return use_balanced<R>(p, H, W, fast_ok) ? p.nwaves : ceil_div(W, WalkShape<R>::SC) * ceil_div(H, 8);
}

template <int R, bool SIGNED, bool SECTOR = false>
void launch_walk_sized(const F32FwdArgs& a, int fast_ok, hipStream_t s) {
    const WalkPlan p = make_walk_plan<R>(a.H, a.W, fast_ok);
    if (use_balanced<R>(p, a.H, a.W, fast_ok)) {
        hipLaunchKernelGGL((k_f32_forward_bal<R, kRRI, kRRE, SIGNED, SECTOR>), dim3(ceil_div(p.nwaves, kWavesPerWG)),
                           dim3(kWGThreads), 0, s, a, p, fast_ok);
    } else {
        launch_walk<R, 8, SIGNED, SECTOR>(a, fast_ok, s);
    }
}

template <int R>
hipError_t launch_radius(const F32FwdArgs& a, hipStream_t s) {
    const int fast_ok = walk_fast_ok(a);
    if (!a.smag) {  // absolute thresholds, no max: classify in the walk
        StageTimer t(CANNY_STAGE_F32_WALK, s);
        if (a.sector)
            launch_walk_sized<R, false, true>(a, fast_ok, s);
        else
            launch_walk_sized<R, false, false>(a, fast_ok, s);
        return hipGetLastError();
    }
    if (!a.maxslots) {  // per-wave slots need no clearing
        StageTimer t(CANNY_STAGE_F32_CLEAR, s);
        hipLaunchKernelGGL(k_f32_clear_max, dim3(1), dim3(kWave), 0, s, a.maxbits);
    }
    {
        StageTimer t(CANNY_STAGE_F32_WALK, s);
        launch_walk_sized<R, true>(a, fast_ok, s);
    }
    if (!a.skip_classify) {
        StageTimer t(CANNY_STAGE_F32_CLASSIFY, s);
        hipLaunchKernelGGL(k_f32_classify, dim3(rows_grid(a.H)), dim3(kRowThreads), 0, s, a);
    }
    return hipGetLastError();
}

}  // namespace

int f32_walk_waves(const F32FwdArgs& a) {
    const int fast_ok = walk_fast_ok(a);
    switch (a.radius) {
        case 1: return walk_waves_r<1>(a.H, a.W, fast_ok);
        case 2: return walk_waves_r<2>(a.H, a.W, fast_ok);
        case 3: return walk_waves_r<3>(a.H, a.W, fast_ok);
        case 4: return walk_waves_r<4>(a.H, a.W, fast_ok);
        case 5: return walk_waves_r<5>(a.H, a.W, fast_ok);
        case 6: return walk_waves_r<6>(a.H, a.W, fast_ok);
        case 7: return walk_waves_r<7>(a.H, a.W, fast_ok);
        case 8: return walk_waves_r<8>(a.H, a.W, fast_ok);
        default: return 0;
    }
}

hipError_t launch_f32_forward(const F32FwdArgs& a, hipStream_t s) {
    switch (a.radius) {
        case 1: return launch_radius<1>(a, s);
        case 2: return launch_radius<2>(a, s);
        case 3: return launch_radius<3>(a, s);
        case 4: return launch_radius<4>(a, s);
        case 5: return launch_radius<5>(a, s);
        case 6: return launch_radius<6>(a, s);
        case 7: return launch_radius<7>(a, s);
        case 8: return launch_radius<8>(a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace canny
