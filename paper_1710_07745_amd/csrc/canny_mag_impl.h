// Differentiable front end of the detector: Steps 1-2 of the paper (Section
// 2.2.1) as a function of the image and the Gaussian scale,
//     M(I, sigma) = sqrt(Gx^2 + Gy^2),  (Gx, Gy) = Sobel * B,  B = G_sigma * I,
// batched over N equal-size images with one sigma per image, replicate
// borders at every stage, and its hand-written adjoint.
//
// Forward (k_mag_fwd): the fp32 strip walk of the float detector up to M.
//
// Backward, given dM = dL/dM (the blurred image is recomputed, not stored):
//   k_mag_bwd_a  recomputes B, Gx, Gy, M per strip, forms
//                dGx = dM Gx / M, dGy = dM Gy / M (0 where M = 0), and applies
//                the transposed Sobel pair, dB = Dx^T Sy^T dGx + Dy^T Sx^T dGy,
//                writing dB to the workspace.
//   k_mag_bwd_b  applies the transposed Gaussian, dT = Gv^T dB and
//                dI = Gh^T dT, and accumulates
//                dL/dsigma = <dT, Gh' I> + <Gv'^T dB, Gh I>
//                (G' = the taps' derivative in sigma) into one partial per wave.
//   k_mag_reduce sums the partials of each image in a fixed order in fp64.
//
// Transposing a 1-D stencil w_k (k = -K..K) applied with clamped reads: the
// adjoint reads the zero-extended source with coefficients w_{-j} at every
// output position except the two edge ones, where the taps that the clamp
// folded onto the edge are gathered back: at position 0 the source at offset
// j >= 0 carries sum_{k <= -j} w_k, at position N-1 the source at offset
// j <= 0 carries sum_{k >= -j} w_k (one position: sum of all taps).
#pragma once

#include "canny_internal.h"
#include "canny_f32_common.h"

namespace canny {
namespace {

constexpr int kMagRows = 32;  // output rows per wave

template <int R>
struct Taps {
    float g[R + 1];      // g_k = g_{-k}
    float dg[R + 1];     // d g_k / d sigma
    float tail[R + 1];   // sum_{k >= j} g_k
    float dtail[R + 1];  // sum_{k >= j} dg_k
};

template <int R>
__device__ __forceinline__ Taps<R> make_taps(float sigma) {
    Taps<R> t;
    float e[R + 1];
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k <= R; ++k) {
        e[k] = expf(-(float)(k * k) / (2.0f * sigma * sigma));
        s += k ? 2.0f * e[k] : e[k];
    }
    float m2 = 0.0f;
#pragma unroll
    for (int k = 0; k <= R; ++k) {
        t.g[k] = e[k] / s;
        m2 += (k ? 2.0f : 1.0f) * t.g[k] * (float)(k * k);
    }
    const float s3 = sigma * sigma * sigma;
#pragma unroll
    for (int k = 0; k <= R; ++k) t.dg[k] = t.g[k] * ((float)(k * k) - m2) / s3;
    t.tail[R] = t.g[R];
    t.dtail[R] = t.dg[R];
#pragma unroll
    for (int k = R - 1; k >= 0; --k) {
        t.tail[k] = t.tail[k + 1] + t.g[k];
        t.dtail[k] = t.dtail[k + 1] + t.dg[k];
    }
    return t;
}

// coefficient of the source at offset j (|j| <= R) for output position p of
// an axis of length n, transposed symmetric taps w with tails tl
template <int R>
__device__ __forceinline__ float tcoef(const float* w, const float* tl, int j, int p, int n) {
    if (n == 1) return j == 0 ? 1.0f * (2.0f * tl[0] - w[0]) : 0.0f;  // all taps
    if (p == 0) return j >= 0 ? tl[j] : 0.0f;
    if (p == n - 1) return j <= 0 ? tl[-j] : 0.0f;
    return w[j < 0 ? -j : j];
}

struct WaveGeom {
    int n, X0, Y0, c0, lane;
    bool ok;
};

template <int HL>
__device__ __forceinline__ WaveGeom wave_geom(int strips_x, int blocks_y, int N) {
    constexpr int SC = 4 * (kWave - 2 * HL);
    WaveGeom w;
    w.lane = threadIdx.x & (kWave - 1);
    const int wave_in_wg = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wg = xcd_remap(blockIdx.x, gridDim.x);
    const int wave = wg * kWavesPerWG + wave_in_wg;
    const int per_img = strips_x * blocks_y;
    w.ok = wave < N * per_img;
    w.n = wave / per_img;
    const int rem = wave - w.n * per_img;
    const int blk = rem / strips_x;
    const int strip = rem - blk * strips_x;
    w.X0 = strip * SC;
    w.Y0 = blk * kMagRows;
    w.c0 = w.X0 - 4 * HL + 4 * w.lane;
    return w;
}

template <int HL>
__device__ __forceinline__ BorderF make_border(int X0, int c0, int W) {
    constexpr int SC = 4 * (kWave - 2 * HL);
    BorderF bd;
    bd.left = X0 == 0;
    bd.right = X0 + SC + 4 * HL > W;
    bd.l0_lane = HL;
    const int off = W - 1 - (X0 - 4 * HL);
    bd.lw_lane = min(off >> 2, kWave - 1);
    bd.lw_px = off & 3;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        bd.outL[k] = c0 + k < 0;
        bd.outR[k] = c0 + k >= W;
    }
    return bd;
}

// midpoint of the values in a row held by the wave (offset that Sobel ignores)
__device__ __forceinline__ float wave_mid(const F4& r0) {
    const float lo = wave_min(fminf(fminf(r0.v[0], r0.v[1]), fminf(r0.v[2], r0.v[3])));
    const float hi = wave_max(fmaxf(fmaxf(r0.v[0], r0.v[1]), fmaxf(r0.v[2], r0.v[3])));
    return bc<float>(__builtin_amdgcn_readfirstlane(bc<int>(0.5f * lo + 0.5f * hi)));
}

// Blur (vertical taps over the window, then horizontal via lane shifts), with
// the blurred row re-extended at the image's left/right edges.
template <int R>
__device__ __forceinline__ F4 blur_row(const F4* win, const float* g, const BorderF& bd) {
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
    return B;
}

// Sobel row terms dx = B(x+1) - B(x-1), sx = B(x-1) + 2B(x) + B(x+1)
__device__ __forceinline__ void sobel_terms(const F4& B, F4& dx, F4& sx) {
    const float bl = from_left_f(B.v[3]), br = from_right_f(B.v[0]);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float xm = k == 0 ? bl : B.v[k - 1];
        const float xp = k == 3 ? br : B.v[k + 1];
        dx.v[k] = xp - xm;
        sx.v[k] = fmaf(2.0f, B.v[k], xm + xp);
    }
}

// push Sobel row terms of row b into 3-row windows, replicating edge rows
__device__ __forceinline__ void push_terms(F4* dxw, F4* sxw, const F4& dx, const F4& sx, int b, int H) {
    dxw[0] = dxw[1]; dxw[1] = dxw[2];
    sxw[0] = sxw[1]; sxw[1] = sxw[2];
    const bool below = b >= H, top = b == 0;
    dxw[2] = sel4(below, dxw[1], dx);
    sxw[2] = sel4(below, sxw[1], sx);
    dxw[1] = sel4(top, dx, dxw[1]);
    sxw[1] = sel4(top, sx, sxw[1]);
    dxw[0] = sel4(top, dx, dxw[0]);
    sxw[0] = sel4(top, sx, sxw[0]);
}

// ------------------------------------------------------------------ forward
template <int R>
__global__ void __launch_bounds__(kWGThreads)
k_mag_fwd(const float* I, const float* sigma, int N, int H, int W, float* M, int strips_x,
          int blocks_y) {
    constexpr int HL = (R + 1 + 3) / 4;
    constexpr int HR = R + 1;
    constexpr int NI = kMagRows + 2 * HR;
    constexpr int PF = 4;
    constexpr int NW = 2 * R + 1 + PF;
    const WaveGeom wg = wave_geom<HL>(strips_x, blocks_y, N);
    if (!wg.ok) return;
    const float* img = I + (int64_t)wg.n * H * W;
    float* out = M + (int64_t)wg.n * H * W;
    const int c0 = wg.c0, X0 = wg.X0, Y0 = wg.Y0;
    const BorderF bd = make_border<HL>(X0, c0, W);
    const bool out_lane = wg.lane >= HL && wg.lane < kWave - HL;
    const Taps<R> tp = make_taps<R>(sigma[wg.n]);
    auto fetch = [&](int i) -> F4 {
        const int y = min(max(Y0 - HR + i, 0), H - 1);
        return load_row_clamped(img + (int64_t)y * W, c0, W);
    };
    F4 win[NW];
#pragma unroll
    for (int k = 0; k < NW; ++k) win[k] = (k >= 2 * R && k - 2 * R < NI) ? fetch(k - 2 * R) : F4{};
    const float off = wave_mid(win[2 * R]);
#pragma unroll
    for (int k = 2 * R; k < NW; ++k)
#pragma unroll
        for (int q = 0; q < 4; ++q) win[k].v[q] -= off;
    F4 dxw[3], sxw[3];
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
        const int b = Y0 - HR + i - R;
        const F4 B = blur_row<R>(win, tp.g, bd);
        F4 dx, sx;
        sobel_terms(B, dx, sx);
        push_terms(dxw, sxw, dx, sx, b, H);
        if (i < 2 * R + 2) continue;
        const int gr = b - 1;  // >= Y0; rows past the image are dropped at the store
        F4 m;
        bool ok[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float gx = fmaf(2.0f, dxw[1].v[k], dxw[0].v[k] + dxw[2].v[k]);
            const float gy = sxw[2].v[k] - sxw[0].v[k];
            m.v[k] = __builtin_amdgcn_sqrtf(fmaf(gx, gx, gy * gy));
            ok[k] = gr < H && out_lane && !bd.outR[k];
        }
        store_row_masked(out + (int64_t)min(gr, H - 1) * W, c0, m, ok);
    }
}

// ------------------------------------------------------------ backward, A
template <int R>
__global__ void __launch_bounds__(kWGThreads)
k_mag_bwd_a(const float* I, const float* sigma, const float* dM, int N, int H, int W, float* dB,
            int strips_x, int blocks_y) {
    constexpr int HL = (R + 2 + 3) / 4;
    constexpr int HR = R + 2;
    constexpr int NI = kMagRows + 2 * HR;
    constexpr int PF = 4;
    constexpr int NW = 2 * R + 1 + PF;
    const WaveGeom wg = wave_geom<HL>(strips_x, blocks_y, N);
    if (!wg.ok) return;
    const int64_t ioff = (int64_t)wg.n * H * W;
    const float* img = I + ioff;
    const float* gm = dM + ioff;
    float* out = dB + ioff;
    const int c0 = wg.c0, X0 = wg.X0, Y0 = wg.Y0;
    const BorderF bd = make_border<HL>(X0, c0, W);
    const bool out_lane = wg.lane >= HL && wg.lane < kWave - HL;
    const Taps<R> tp = make_taps<R>(sigma[wg.n]);
    auto fetch = [&](int i) -> F4 {
        const int y = min(max(Y0 - HR + i, 0), H - 1);
        return load_row_clamped(img + (int64_t)y * W, c0, W);
    };
    F4 win[NW];
#pragma unroll
    for (int k = 0; k < NW; ++k) win[k] = (k >= 2 * R && k - 2 * R < NI) ? fetch(k - 2 * R) : F4{};
    const float off = wave_mid(win[2 * R]);
#pragma unroll
    for (int k = 2 * R; k < NW; ++k)
#pragma unroll
        for (int q = 0; q < 4; ++q) win[k].v[q] -= off;
    bool inimg[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) inimg[k] = !bd.outL[k] && !bd.outR[k];
    // dM row consumed at iteration i (i >= 2R + 2), loaded GD iterations
    // earlier into a ring (compile-time slots in the unrolled loop)
    constexpr int GD = 4;
    auto gm_row = [&](int i) -> F4 {
        const int gr = Y0 - HR + i - R - 1;
        return load_row_clamped(gm + (int64_t)min(max(gr, 0), H - 1) * W, c0, W);
    };
    F4 gq[GD];
#pragma unroll
    for (int j = 2 * R + 2; j < GD && j < NI; ++j) gq[j % GD] = gm_row(j);  // due before iteration 0
    F4 dxw[3], sxw[3];
    F4 gxw[3], vw[3];  // rows gr-2 .. gr of dGx and of v = Sx^T dGy
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        F4 gmv = {};
        if (i >= 2 * R + 2) gmv = gq[i % GD];
        if (i + GD >= 2 * R + 2 && i + GD < NI) gq[(i + GD) % GD] = gm_row(i + GD);  // i + GD >= GD
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
        const int b = Y0 - HR + i - R;
        const F4 B = blur_row<R>(win, tp.g, bd);
        F4 dx, sx;
        sobel_terms(B, dx, sx);
        push_terms(dxw, sxw, dx, sx, b, H);
        if (i < 2 * R + 2) continue;

        // dG of row gr (zero outside the image: the adjoint reads it zero-extended)
        const int gr = b - 1;
        const bool row_in = gr >= 0 && gr < H;
        F4 dgx, dgy;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float gx = fmaf(2.0f, dxw[1].v[k], dxw[0].v[k] + dxw[2].v[k]);
            const float gy = sxw[2].v[k] - sxw[0].v[k];
            const float m = __builtin_amdgcn_sqrtf(fmaf(gx, gx, gy * gy));
            const bool live = row_in && inimg[k] && m > 0.0f;
            const float q = live ? gmv.v[k] * __builtin_amdgcn_rcpf(m) : 0.0f;
            dgx.v[k] = q * gx;
            dgy.v[k] = q * gy;
        }
        // v = Sx^T dGy along the row
        F4 v;
        {
            const float l = from_left_f(dgy.v[3]), r = from_right_f(dgy.v[0]);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const float xm = k == 0 ? l : dgy.v[k - 1];
                const float xp = k == 3 ? r : dgy.v[k + 1];
                const int x = c0 + k;
                float val = xm + xp + 2.0f * dgy.v[k];
                if (bd.left || bd.right) {
                    if (W == 1) val = 4.0f * dgy.v[k];
                    else if (x == 0) val = 3.0f * dgy.v[k] + xp;
                    else if (x == W - 1) val = 3.0f * dgy.v[k] + xm;
                }
                v.v[k] = val;
            }
        }
        gxw[0] = gxw[1]; gxw[1] = gxw[2]; gxw[2] = dgx;
        vw[0] = vw[1]; vw[1] = vw[2]; vw[2] = v;
        if (i < 2 * R + 4) continue;

        // dB of row db = gr - 1 from dG rows db-1, db, db+1 (db >= Y0; rows
        // past the image are dropped at the store)
        const int db = gr - 1;
        F4 u, w;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            float uu = gxw[0].v[k] + gxw[2].v[k] + 2.0f * gxw[1].v[k];  // Sy^T
            float ww = vw[0].v[k] - vw[2].v[k];                          // Dy^T
            if (H == 1) {
                uu = 4.0f * gxw[1].v[k];
                ww = 0.0f;
            } else if (db == 0) {
                uu = 3.0f * gxw[1].v[k] + gxw[2].v[k];
                ww = -vw[1].v[k] - vw[2].v[k];
            } else if (db == H - 1) {
                uu = 3.0f * gxw[1].v[k] + gxw[0].v[k];
                ww = vw[1].v[k] + vw[0].v[k];
            }
            u.v[k] = uu;
            w.v[k] = ww;
        }
        const float ul = from_left_f(u.v[3]), ur = from_right_f(u.v[0]);
        F4 res;
        bool ok[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float xm = k == 0 ? ul : u.v[k - 1];
            const float xp = k == 3 ? ur : u.v[k + 1];
            const int x = c0 + k;
            float dxu = xm - xp;  // Dx^T
            if (bd.left || bd.right) {
                if (W == 1) dxu = 0.0f;
                else if (x == 0) dxu = -u.v[k] - xp;
                else if (x == W - 1) dxu = u.v[k] + xm;
            }
            res.v[k] = dxu + w.v[k];
            ok[k] = db < H && out_lane && !bd.outR[k];
        }
        store_row_masked(out + (int64_t)min(db, H - 1) * W, c0, res, ok);
    }
}

// ------------------------------------------------------------ backward, B
template <int R>
__global__ void __launch_bounds__(kWGThreads)
k_mag_bwd_b(const float* I, const float* sigma, const float* dB, int N, int H, int W, float* dI,
            float* partial, int strips_x, int blocks_y) {
    constexpr int HL = (R + 3) / 4;
    constexpr int NI = kMagRows + 2 * R;
    constexpr int PF = 4;
    constexpr int NW = 2 * R + 1 + PF;
    const WaveGeom wg = wave_geom<HL>(strips_x, blocks_y, N);
    if (!wg.ok) return;
    const int64_t ioff = (int64_t)wg.n * H * W;
    const float* img = I + ioff;
    const float* src = dB + ioff;
    float* out = dI + ioff;
    const int c0 = wg.c0, X0 = wg.X0, Y0 = wg.Y0;
    const BorderF bd = make_border<HL>(X0, c0, W);
    const bool out_lane = wg.lane >= HL && wg.lane < kWave - HL;
    const Taps<R> tp = make_taps<R>(sigma[wg.n]);
    bool inimg[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) inimg[k] = !bd.outL[k] && !bd.outR[k];
    // dB rows Y0-R+i, zero outside the image (out-of-range loads read 0, so
    // every row issues the same loads)
    auto fetch = [&](int i) -> F4 {
        const int y = Y0 - R + i;
        const bool row_in = y >= 0 && y < H;
        bool ok[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) ok[k] = row_in && inimg[k];
        return load_row_masked(src + (int64_t)min(max(y, 0), H - 1) * W, c0, ok);
    };
    // input row of output row y = Y0 - 2R + i, consumed at iteration i >= 2R,
    // loaded GD iterations earlier into a ring
    constexpr int GD = 4;
    auto in_row = [&](int i) -> F4 {
        const int y = Y0 - 2 * R + i;
        return load_row_clamped(img + (int64_t)min(y, H - 1) * W, c0, W);
    };
    F4 iq[GD];
#pragma unroll
    for (int j = 2 * R; j < GD && j < NI; ++j) iq[j % GD] = in_row(j);  // due before iteration 0
    F4 win[NW];
#pragma unroll
    for (int k = 0; k < NW; ++k) win[k] = (k >= 2 * R && k - 2 * R < NI) ? fetch(k - 2 * R) : F4{};
    float acc = 0.0f;
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        F4 Ir = {};
        if (i >= 2 * R) Ir = iq[i % GD];
        if (i + GD >= 2 * R && i + GD < NI) iq[(i + GD) % GD] = in_row(i + GD);  // i + GD >= GD
        if (i > 0) {
#pragma unroll
            for (int k = 0; k < NW - 1; ++k) win[k] = win[k + 1];
            if (i + PF < NI) win[NW - 1] = fetch(i + PF);
        }
        if (i < 2 * R) continue;
        const int y = Y0 - R + i - R;  // output row (>= Y0); rows past the image are dropped
        const bool row_ok = y < H;
        // dT = Gv^T dB and dT' = Gv'^T dB at row y
        F4 dT, dTp;
        const bool edge_row = y == 0 || y == H - 1;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            float a0, a1;
            if (!edge_row) {
                a0 = tp.g[0] * win[R].v[k];
                a1 = tp.dg[0] * win[R].v[k];
#pragma unroll
                for (int j = 1; j <= R; ++j) {
                    const float s2 = win[R - j].v[k] + win[R + j].v[k];
                    a0 = fmaf(tp.g[j], s2, a0);
                    a1 = fmaf(tp.dg[j], s2, a1);
                }
            } else {
                a0 = 0.0f;
                a1 = 0.0f;
#pragma unroll
                for (int j = -R; j <= R; ++j) {
                    a0 = fmaf(tcoef<R>(tp.g, tp.tail, j, y, H), win[R + j].v[k], a0);
                    a1 = fmaf(tcoef<R>(tp.dg, tp.dtail, j, y, H), win[R + j].v[k], a1);
                }
            }
            dT.v[k] = a0;
            dTp.v[k] = a1;
        }
        // T = Gh I and T' = Gh' I of the input row y (clamped reads, Ir above)
        float ext[4 + 2 * R];
#pragma unroll
        for (int e = -R; e < 4 + R; ++e) ext[e + R] = lane_ext(Ir, e);
        // dI = Gh^T dT (dT is zero outside the image's columns)
        float dext[4 + 2 * R];
#pragma unroll
        for (int e = -R; e < 4 + R; ++e) dext[e + R] = lane_ext(dT, e);
        F4 res;
        bool ok[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            float t0 = tp.g[0] * ext[k + R], t1 = tp.dg[0] * ext[k + R];
#pragma unroll
            for (int j = 1; j <= R; ++j) {
                const float s2 = ext[k + R - j] + ext[k + R + j];
                t0 = fmaf(tp.g[j], s2, t0);
                t1 = fmaf(tp.dg[j], s2, t1);
            }
            const int x = c0 + k;
            float di;
            if ((bd.left || bd.right) && (x == 0 || x == W - 1)) {
                di = 0.0f;
#pragma unroll
                for (int j = -R; j <= R; ++j) di = fmaf(tcoef<R>(tp.g, tp.tail, j, x, W), dext[k + R + j], di);
            } else {
                di = tp.g[0] * dext[k + R];
#pragma unroll
                for (int j = 1; j <= R; ++j) di = fmaf(tp.g[j], dext[k + R - j] + dext[k + R + j], di);
            }
            res.v[k] = di;
            ok[k] = row_ok && out_lane && inimg[k];
            acc = ok[k] ? fmaf(dT.v[k], t1, fmaf(dTp.v[k], t0, acc)) : acc;
        }
        store_row_masked(out + (int64_t)min(y, H - 1) * W, c0, res, ok);
    }
    // fixed-order wave reduction of the dsigma partial
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o);
    if (wg.lane == 0) {
        const int per_img = strips_x * blocks_y;
        const int wave = wg.n * per_img + (wg.Y0 / kMagRows) * strips_x +
                         wg.X0 / (4 * (kWave - 2 * HL));
        partial[wave] = acc;
    }
}

__global__ void __launch_bounds__(kWGThreads) __attribute__((unused))
k_mag_reduce(const float* partial, int per_img, float* dsigma) {
    __shared__ double s[kWGThreads];
    const int n = blockIdx.x;
    double a = 0.0;
    for (int i = threadIdx.x; i < per_img; i += kWGThreads) a += (double)partial[(int64_t)n * per_img + i];
    s[threadIdx.x] = a;
    __syncthreads();
    for (int w = kWGThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) dsigma[n] = (float)s[0];
}

struct Grid {
    int strips_x, blocks_y, nwg, per_img;
};

template <int HL>
Grid grid_for(int N, int H, int W) {
    constexpr int SC = 4 * (kWave - 2 * HL);
    Grid g;
    g.strips_x = ceil_div(W, SC);
    g.blocks_y = ceil_div(H, kMagRows);
    g.per_img = g.strips_x * g.blocks_y;
    g.nwg = (int)ceil_div64((int64_t)N * g.per_img, kWavesPerWG);
    return g;
}

template <int R>
hipError_t fwd_r(const float* I, const float* sigma, int N, int H, int W, float* M, hipStream_t s) {
    constexpr int HL = (R + 1 + 3) / 4;
    const Grid g = grid_for<HL>(N, H, W);
    hipLaunchKernelGGL(k_mag_fwd<R>, dim3(g.nwg), dim3(kWGThreads), 0, s, I, sigma, N, H, W, M,
                       g.strips_x, g.blocks_y);
    return hipGetLastError();
}

template <int R>
hipError_t bwd_r(const float* I, const float* sigma, const float* dM, int N, int H, int W, float* dI,
                 float* dsigma, float* dB, float* partial, hipStream_t s) {
    constexpr int HLA = (R + 2 + 3) / 4, HLB = (R + 3) / 4;
    const Grid ga = grid_for<HLA>(N, H, W), gb = grid_for<HLB>(N, H, W);
    hipLaunchKernelGGL(k_mag_bwd_a<R>, dim3(ga.nwg), dim3(kWGThreads), 0, s, I, sigma, dM, N, H, W, dB,
                       ga.strips_x, ga.blocks_y);
    hipLaunchKernelGGL(k_mag_bwd_b<R>, dim3(gb.nwg), dim3(kWGThreads), 0, s, I, sigma, dB, N, H, W, dI,
                       partial, gb.strips_x, gb.blocks_y);
    hipLaunchKernelGGL(k_mag_reduce, dim3(N), dim3(kWGThreads), 0, s, partial, gb.per_img, dsigma);
    return hipGetLastError();
}

}  // namespace

// Radius groups compiled in separate translation units (the unrolled row
// loops make each radius a large compile); each returns
// hipErrorInvalidValue for a radius outside its group.
#define CANNY_MAG_GROUP_DECL(g)                                                                   \
    hipError_t mag_forward_g##g(const float* I, const float* sigma, int N, int H, int W, int radius, \
                                float* M, hipStream_t s);                                        \
    hipError_t mag_backward_g##g(const float* I, const float* sigma, const float* dM, int N, int H,  \
                                 int W, int radius, float* dI, float* dsigma, float* dB,           \
                                 float* partial, hipStream_t s);
CANNY_MAG_GROUP_DECL(1)
CANNY_MAG_GROUP_DECL(2)
CANNY_MAG_GROUP_DECL(3)
CANNY_MAG_GROUP_DECL(4)
CANNY_MAG_GROUP_DECL(5)
CANNY_MAG_GROUP_DECL(6)
#undef CANNY_MAG_GROUP_DECL

}  // namespace canny
