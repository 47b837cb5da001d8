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
// can be classified, so there are two launches: pass A runs the walk up to M
// and reduces max(Gx^2 + Gy^2) into one word (atomicMax on the float bits,
// order-independent because the value is non-negative); pass B runs the full
// walk and derives the thresholds from that word on the device.
//
// Accuracy: every stage before the strength is linear, and Sobel ignores a
// constant offset, so the walk filters X - c instead of X, with c the
// midpoint of the image's value range (min and max are reduced in pass A;
// without pass A, the midpoint of the wave's first input row).  That halves
// the magnitude the fp32 accumulations round at, and a constant image gives
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

template <int R, int RR, bool PASS_B>
__global__ void __launch_bounds__(kWGThreads)
k_f32_forward(F32FwdArgs a, int strips_x, int nwaves, int fast_ok) {
    constexpr int HL = (R + 2 + 3) / 4;  // halo lanes per side
    constexpr int SC = 4 * (kWave - 2 * HL);
    constexpr int HR = R + 2;            // halo rows per side
    constexpr int NI = PASS_B ? RR + 2 * HR : RR + 2 * HR - 1;
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

    float lo = a.low, hi = a.high;
    if (PASS_B && (a.relative || a.max_out)) {
        const float mx = sqrtf(bc<float>(*a.maxbits));
        if (a.relative) {
            lo = a.low * mx;
            hi = a.high * mx;
        }
        if (a.max_out && wave == 0 && lane == 0) *a.max_out = mx;
    }

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
    if (PASS_B && a.use_range) {
        off = 0.5f * ord2f(a.maxbits[1]) + 0.5f * ord2f(a.maxbits[2]);
    } else {
        const F4& r0 = win[2 * R];
        const float lo = wave_min(fminf(fminf(r0.v[0], r0.v[1]), fminf(r0.v[2], r0.v[3])));
        const float hi = wave_max(fmaxf(fmaxf(r0.v[0], r0.v[1]), fmaxf(r0.v[2], r0.v[3])));
        off = 0.5f * lo + 0.5f * hi;
    }
    off = bc<float>(__builtin_amdgcn_readfirstlane(bc<int>(off)));  // wave-uniform
    float xmin = 3.402823466e38f, xmax = -3.402823466e38f;  // pass A: input range
#pragma unroll
    for (int k = 2 * R; k < NW; ++k) {
        if (k - 2 * R < NI) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (!PASS_B) { xmin = fminf(xmin, win[k].v[q]); xmax = fmaxf(xmax, win[k].v[q]); }
                win[k].v[q] -= off;
            }
        }
    }

    F4 dxw[3], sxw[3];
    MRowF mw[3];
    F4 gxp, gyp, gxc, gyc;  // gradients of rows g-1 (prev) and g (cur)
    float smax = 0.0f;

#pragma unroll
    for (int i = 0; i < NI; ++i) {
        if (i > 0) {
#pragma unroll
            for (int k = 0; k < NW - 1; ++k) win[k] = win[k + 1];
            if (i + PF < NI) {
                win[NW - 1] = fetch(i + PF);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (!PASS_B) {
                        xmin = fminf(xmin, win[NW - 1].v[q]);
                        xmax = fmaxf(xmax, win[NW - 1].v[q]);
                    }
                    win[NW - 1].v[q] -= off;
                }
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
        if (!PASS_B) {
            if (gr >= Y0 && gr < Y0 + RR && gr < H && out_lane) {
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (!bd.outR[k]) smax = fmaxf(smax, s.v[k]);
            }
            continue;
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
            const uint32_t code = (keep && mc > hi) ? 2u : ((keep && mc >= lo) ? 1u : 0u);
            if (!bd.outR[k]) byte |= code << (2 * k);
        }
        if (out_lane && c0 < W) {
            a.cls[(int64_t)n * a.cpitch + (c0 >> 2)] = (uint8_t)byte;
            if (a.mag) {
                float* mrow = a.mag + (int64_t)n * W;
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (!bd.outR[k]) mrow[c0 + k] = c.c[k];
            }
        }
    }

    if (!PASS_B) {
        uint32_t v = bc<uint32_t>(smax);
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o));
        const float wmin = wave_min(xmin), wmax = wave_max(xmax);
        if (lane == 0) {
            if (v) atomicMax(a.maxbits, v);
            atomicMin(a.maxbits + 1, f2ord(wmin));
            atomicMax(a.maxbits + 2, f2ord(wmax));
        }
    }
}

// resets the max-pass words: max M^2 = 0, min code = all ones, max code = 0
__global__ void k_reset_range(uint32_t* p) {
    p[0] = 0u;
    p[1] = 0xFFFFFFFFu;
    p[2] = 0u;
}

template <int R>
hipError_t launch_radius(const F32FwdArgs& a, hipStream_t s) {
    constexpr int RR = 32;
    constexpr int HL = (R + 2 + 3) / 4;
    constexpr int SC = 4 * (kWave - 2 * HL);
    const int strips_x = ceil_div(a.W, SC);
    const int nwaves = strips_x * ceil_div(a.H, RR);
    const int nwg = ceil_div(nwaves, kWavesPerWG);
    const int fast_ok = ((uintptr_t)a.in % 16 == 0) && (a.pitch % 4 == 0);
    if (a.relative || a.max_out) {
        hipLaunchKernelGGL(k_reset_range, dim3(1), dim3(1), 0, s, a.maxbits);
        hipLaunchKernelGGL((k_f32_forward<R, RR, false>), dim3(nwg), dim3(kWGThreads), 0, s, a,
                           strips_x, nwaves, fast_ok);
    }
    hipLaunchKernelGGL((k_f32_forward<R, RR, true>), dim3(nwg), dim3(kWGThreads), 0, s, a,
                       strips_x, nwaves, fast_ok);
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
