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
// requested) the path is: a memory-bound min/max pass over the input, the
// walk with a threshold-free epilogue that stores the strength with its sign
// carrying the suppression decision (+M kept, -M suppressed) and reduces the
// largest M into one word (atomicMax on the float bits, order-independent
// because the value is non-negative), then an elementwise pass that derives
// the thresholds from that word and writes the class map.  The walk, the
// expensive part, therefore runs once per image in both cases.
//
// Accuracy: every stage before the strength is linear, and Sobel ignores a
// constant offset, so the walk filters X - c instead of X, with c the
// midpoint of the image's value range (from the min/max pass; without it,
// the midpoint of the wave's first input row).  That halves the magnitude
// the fp32 accumulations round at, and a constant image gives exactly zero.
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
#include "canny.h"
#include "canny_internal.h"
#include "canny_f32_common.h"

namespace canny {
namespace {

struct MRowF {
    float c[4];
    float l, r;  // column c0-1 and c0+4
};

__device__ __forceinline__ float lerpf_(float p, float d, float t) { return fmaf(t, d - p, p); }

__device__ __forceinline__ MRowF selm(bool p, const MRowF& a, const MRowF& b) {
    MRowF r;
#pragma unroll
    for (int k = 0; k < 4; ++k) r.c[k] = p ? a.c[k] : b.c[k];
    r.l = p ? a.l : b.l;
    r.r = p ? a.r : b.r;
    return r;
}

template <int R, int RR, bool SIGNED>
__global__ void __launch_bounds__(kWGThreads)
k_f32_forward(F32FwdArgs a, int strips_x, int nwaves, int fast_ok) {
    constexpr int HL = (R + 2 + 3) / 4;  // halo lanes per side
    constexpr int SC = 4 * (kWave - 2 * HL);
    constexpr int HR = R + 2;            // halo rows per side
    constexpr int NI = RR + 2 * HR;
    constexpr int PF = 4;                // rows loaded ahead

    const int lane = threadIdx.x & (kWave - 1);
    const int wave_in_wg = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wg = xcd_remap(blockIdx.x, gridDim.x);
    const int wave = wg * kWavesPerWG + wave_in_wg;
    if (wave >= nwaves) return;
    const int strip = wave % strips_x;
    const int blk = wave / strips_x;
    const int X0 = strip * SC;
    const int Y0 = blk * RR;
    const int H = a.H, W = a.W;
    const int c0 = X0 - 4 * HL + 4 * lane;

    BorderF bd;
    bd.left = X0 == 0;
    bd.right = X0 + SC + 4 * HL > W;
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
    const bool fast = fast_ok && c0 >= 0 && c0 + 4 <= W;

    float g[R + 1];
#pragma unroll
    for (int j = 0; j <= R; ++j) g[j] = a.g[j];

    const float lo = a.low, hi = a.high;  // absolute thresholds (direct epilogue)

    // rolling window: win[0..2R] are input rows vi-2R .. vi, win[2R+1..] are
    // rows loaded PF ahead
    constexpr int NW = 2 * R + 1 + PF;
    auto fetch = [&](int i) -> F4 {
        const int y = min(max(Y0 - HR + i, 0), H - 1);
        return load_row(a.in + (int64_t)y * a.pitch, c0, W, fast);
    };
    F4 win[NW];
#pragma unroll
    for (int k = 0; k < NW; ++k) win[k] = (k >= 2 * R && k - 2 * R < NI) ? fetch(k - 2 * R) : F4{};

    // offset c subtracted from every input value (see the file comment)
    float off;
    if (SIGNED) {  // image range from the min/max pass's per-workgroup partials
        float lo = 3.402823466e38f, hi = -3.402823466e38f;
        for (int j = lane; j < a.nrange; j += kWave) {
            const float2 p = a.range[j];
            lo = fminf(lo, p.x);
            hi = fmaxf(hi, p.y);
        }
        off = 0.5f * wave_min(lo) + 0.5f * wave_max(hi);
    } else {
        const F4& r0 = win[2 * R];
        const float lo = wave_min(fminf(fminf(r0.v[0], r0.v[1]), fminf(r0.v[2], r0.v[3])));
        const float hi = wave_max(fmaxf(fmaxf(r0.v[0], r0.v[1]), fmaxf(r0.v[2], r0.v[3])));
        off = 0.5f * lo + 0.5f * hi;
    }
    off = bc<float>(__builtin_amdgcn_readfirstlane(bc<int>(off)));  // wave-uniform
#pragma unroll
    for (int k = 2 * R; k < NW; ++k) {
        if (k - 2 * R < NI) {
#pragma unroll
            for (int q = 0; q < 4; ++q) win[k].v[q] -= off;
        }
    }

    F4 dxw[3], sxw[3];
    MRowF mw[3];
    F4 gxp, gyp, gxc, gyc;  // gradients of rows g-1 (prev) and g (cur)
    float mmax = 0.0f;  // largest M of the rows this wave outputs

#pragma unroll
    for (int i = 0; i < NI; ++i) {
        if (i > 0) {
#pragma unroll
            for (int k = 0; k < NW - 1; ++k) win[k] = win[k + 1];
            if (i + PF < NI) {
                win[NW - 1] = fetch(i + PF);
#pragma unroll
                for (int q = 0; q < 4; ++q) win[NW - 1].v[q] -= off;
            }
        }
        if (i < 2 * R) continue;
        // ---- Step 1: Gaussian, row b = vi - R (vertical taps, then horizontal)
        const int b = Y0 - HR + i - R;
        F4 V;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            float acc = g[0] * win[R].v[k];
#pragma unroll
            for (int j = 1; j <= R; ++j) acc = fmaf(g[j], win[R - j].v[k] + win[R + j].v[k], acc);
            V.v[k] = acc;
        }
        float ext[4 + 2 * R];
#pragma unroll
        for (int e = -R; e < 4 + R; ++e) ext[e + R] = lane_ext(V, e);
        F4 B;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            float acc = g[0] * ext[k + R];
#pragma unroll
            for (int j = 1; j <= R; ++j) acc = fmaf(g[j], ext[k + R - j] + ext[k + R + j], acc);
            B.v[k] = acc;
        }
        fix_cols(B, bd);
        // ---- Step 2a: Sobel row terms
        const float bl = from_left_f(B.v[3]), br = from_right_f(B.v[0]);
        F4 dx, sx;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float xm = k == 0 ? bl : B.v[k - 1];
            const float xp = k == 3 ? br : B.v[k + 1];
            dx.v[k] = xp - xm;
            sx.v[k] = fmaf(2.0f, B.v[k], xm + xp);
        }
        dxw[0] = dxw[1]; dxw[1] = dxw[2];
        sxw[0] = sxw[1]; sxw[1] = sxw[2];
        const bool below = b >= H, top = b == 0;  // rows outside replicate the edge row
        dxw[2] = sel4(below, dxw[1], dx);
        sxw[2] = sel4(below, sxw[1], sx);
        dxw[1] = sel4(top, dx, dxw[1]);
        sxw[1] = sel4(top, sx, sxw[1]);
        dxw[0] = sel4(top, dx, dxw[0]);
        sxw[0] = sel4(top, sx, sxw[0]);
        if (i < 2 * R + 2) continue;

        // ---- Step 2b: gradients and strength of row gr = b - 1
        const int gr = b - 1;
        F4 gx, gy, s;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            gx.v[k] = fmaf(2.0f, dxw[1].v[k], dxw[0].v[k] + dxw[2].v[k]);
            gy.v[k] = sxw[2].v[k] - sxw[0].v[k];
            s.v[k] = fmaf(gx.v[k], gx.v[k], gy.v[k] * gy.v[k]);
        }
        gxp = gxc; gyp = gyc;
        gxc = gx; gyc = gy;
        F4 M;
#pragma unroll
        for (int k = 0; k < 4; ++k) M.v[k] = sqrtf(s.v[k]);
        fix_cols(M, bd);
        MRowF m;
#pragma unroll
        for (int k = 0; k < 4; ++k) m.c[k] = M.v[k];
        m.l = from_left_f(M.v[3]);
        m.r = from_right_f(M.v[0]);
        mw[0] = mw[1]; mw[1] = mw[2];
        mw[2] = selm(gr >= H, mw[1], m);
        mw[1] = selm(gr == 0, m, mw[1]);
        mw[0] = selm(gr == 0, m, mw[0]);
        if (i < 2 * R + 4) continue;

        // ---- Step 3 + thresholds: row n = gr - 1
        const int n = gr - 1;
        if (n < Y0 || n >= H) continue;
        const MRowF& u = mw[0];
        const MRowF& c = mw[1];
        const MRowF& d = mw[2];
        uint32_t byte = 0;
        F4 sv;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float mc = c.c[k];
            const float cl = k == 0 ? c.l : c.c[k - 1], cr = k == 3 ? c.r : c.c[k + 1];
            const float ul = k == 0 ? u.l : u.c[k - 1], uc = u.c[k], ur = k == 3 ? u.r : u.c[k + 1];
            const float dl = k == 0 ? d.l : d.c[k - 1], dc = d.c[k], dr = k == 3 ? d.r : d.c[k + 1];
            const float gxk = gxp.v[k], gyk = gyp.v[k];
            const float ax = fabsf(gxk), ay = fabsf(gyk);
            const bool domx = ax >= ay;
            const bool same = gxk * gyk > 0.0f;
            const float mn = fminf(ax, ay), mxv = fmaxf(ax, ay);
            const float t = mxv > 0.0f ? mn * __builtin_amdgcn_rcpf(mxv) : 0.0f;
            const float fp = domx ? cr : dc;
            const float fd = same ? dr : (domx ? ur : dl);
            const float bp = domx ? cl : uc;
            const float bdg = same ? ul : (domx ? dl : ur);
            const float ahead = lerpf_(fp, fd, t);
            const float behind = lerpf_(bp, bdg, t);
            const bool keep = mc > 0.0f && mc > behind && mc >= ahead;
            if (SIGNED) {
                sv.v[k] = keep ? mc : -mc;
                if (!bd.outR[k]) mmax = fmaxf(mmax, mc);
            } else {
                const uint32_t code = (keep && mc > hi) ? 2u : ((keep && mc >= lo) ? 1u : 0u);
                if (!bd.outR[k]) byte |= code << (2 * k);
            }
        }
        if (out_lane && c0 < W) {
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
                        if (!bd.outR[k]) mrow[c0 + k] = c.c[k];
                }
            }
        }
    }

    if (SIGNED) {
        const float wmax = out_lane ? mmax : 0.0f;
        const uint32_t v = bc<uint32_t>(wave_max(wmax));
        if (lane == 0 && v) atomicMax(a.maxbits, v);
    }
}

constexpr int kRowThreads = 256;  // one workgroup walks whole rows
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Input min and max, one (min, max) pair per workgroup written to
// a.range[blockIdx.x] (no atomics: the walk reduces the pairs itself).
// Workgroup b takes rows b, b + gridDim.x, ...; each thread takes float4
// quads of a row.  Also clears the largest-strength word the walk reduces
// into, which is safe because the walk is launched after this kernel.
__global__ void __launch_bounds__(kRowThreads)
k_f32_minmax(F32FwdArgs a, int quads_ok) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *a.maxbits = 0u;
    float lo = 3.402823466e38f, hi = -3.402823466e38f;
    const int W = a.W;
    const int nq = W >> 2;
    for (int y = blockIdx.x; y < a.H; y += gridDim.x) {
        const float* row = a.in + (int64_t)y * a.pitch;
        int x0 = 0;
        if (quads_ok) {
            const f32x4* r4 = reinterpret_cast<const f32x4*>(row);
            for (int q = threadIdx.x; q < nq; q += kRowThreads) {
                const f32x4 v = r4[q];
                lo = fminf(lo, fminf(fminf(v.x, v.y), fminf(v.z, v.w)));
                hi = fmaxf(hi, fmaxf(fmaxf(v.x, v.y), fmaxf(v.z, v.w)));
            }
            x0 = 4 * nq;
        }
        for (int x = x0 + threadIdx.x; x < W; x += kRowThreads) {
            lo = fminf(lo, row[x]);
            hi = fmaxf(hi, row[x]);
        }
    }
    __shared__ float2 part[kRowThreads / kWave];
    lo = wave_min(lo);
    hi = wave_max(hi);
    const int wv = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) part[wv] = make_float2(lo, hi);
    __syncthreads();
    if (threadIdx.x == 0) {
        float2 r = part[0];
        for (int k = 1; k < kRowThreads / kWave; ++k) {
            r.x = fminf(r.x, part[k].x);
            r.y = fmaxf(r.y, part[k].y);
        }
        a.range[blockIdx.x] = r;
    }
}

// Thresholds and classes from the signed strength map: a pixel is kept iff
// its stored value is positive (M > 0 and not suppressed); then strong iff
// M > high, weak iff M >= low, with low/high scaled by the largest M when
// thresholds are relative.  Each thread packs 16 pixels into one 32-bit
// word of the class map.
__global__ void __launch_bounds__(kRowThreads)
k_f32_classify(F32FwdArgs a) {
    const float mx = bc<float>(a.maxbits[0]);
    const float lo = a.relative ? a.low * mx : a.low;
    const float hi = a.relative ? a.high * mx : a.high;
    if (a.max_out && blockIdx.x == 0 && threadIdx.x == 0) *a.max_out = mx;
    const int W = a.W;
    const int nq = (W + 3) >> 2;     // quads of the row (pitch holds them all)
    const int nw = (nq + 3) >> 2;    // 16-pixel words
    const bool mag4 = a.mag && (W % 4 == 0) && ((uintptr_t)a.mag % 16 == 0);
    for (int y = blockIdx.x; y < a.H; y += gridDim.x) {
        const float* srow = a.smag + (int64_t)y * a.spitch;
        uint32_t* crow = reinterpret_cast<uint32_t*>(a.cls + (int64_t)y * a.cpitch);
        for (int w = threadIdx.x; w < nw; w += kRowThreads) {
            uint32_t word = 0;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int q = 4 * w + j;
                if (q >= nq) break;
                const f32x4 v4 = reinterpret_cast<const f32x4*>(srow)[q];
                const float v[4] = {v4.x, v4.y, v4.z, v4.w};
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int x = 4 * q + k;
                    const uint32_t code = (x < W && v[k] > 0.0f) ? (v[k] > hi ? 2u : (v[k] >= lo ? 1u : 0u)) : 0u;
                    word |= code << (8 * j + 2 * k);
                }
                if (a.mag) {
                    float* mrow = a.mag + (int64_t)y * W;
                    if (mag4) {
                        *reinterpret_cast<float4*>(mrow + 4 * q) =
                            make_float4(fabsf(v[0]), fabsf(v[1]), fabsf(v[2]), fabsf(v[3]));
                    } else {
#pragma unroll
                        for (int k = 0; k < 4; ++k)
                            if (4 * q + k < W) mrow[4 * q + k] = fabsf(v[k]);
                    }
                }
            }
            crow[w] = word;
        }
    }
}

int rows_grid(int H) { return min(H, 8 * 256); }

template <int R>
hipError_t launch_radius(const F32FwdArgs& a, hipStream_t s) {
    constexpr int RR = 32;
    constexpr int HL = (R + 2 + 3) / 4;
    constexpr int SC = 4 * (kWave - 2 * HL);
    const int strips_x = ceil_div(a.W, SC);
    const int nwaves = strips_x * ceil_div(a.H, RR);
    const int nwg = ceil_div(nwaves, kWavesPerWG);
    const int fast_ok = ((uintptr_t)a.in % 16 == 0) && (a.pitch % 4 == 0);
    if (!a.smag) {  // absolute thresholds, no max: classify in the walk
        StageTimer t(CANNY_STAGE_F32_WALK, s);
        hipLaunchKernelGGL((k_f32_forward<R, RR, false>), dim3(nwg), dim3(kWGThreads), 0, s, a,
                           strips_x, nwaves, fast_ok);
        return hipGetLastError();
    }
    F32FwdArgs b = a;
    b.nrange = min(a.H, kF32RangeParts);
    {
        StageTimer t(CANNY_STAGE_F32_MINMAX, s);
        hipLaunchKernelGGL(k_f32_minmax, dim3(b.nrange), dim3(kRowThreads), 0, s, b, fast_ok);
    }
    {
        StageTimer t(CANNY_STAGE_F32_WALK, s);
        hipLaunchKernelGGL((k_f32_forward<R, RR, true>), dim3(nwg), dim3(kWGThreads), 0, s, b,
                           strips_x, nwaves, fast_ok);
    }
    {
        StageTimer t(CANNY_STAGE_F32_CLASSIFY, s);
        hipLaunchKernelGGL(k_f32_classify, dim3(rows_grid(a.H)), dim3(kRowThreads), 0, s, b);
    }
    return hipGetLastError();
}

}  // namespace

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
