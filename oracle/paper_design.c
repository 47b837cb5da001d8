/*
 * paper_design.c -- the float Canny operator on the CPU in the paper's own
 * parallel design, as a measured baseline.
 *
 * TEST AND BENCHMARK INFRASTRUCTURE ONLY, like the oracle beside it: only the
 * test suite and the CPU leg of the benchmark load it; the HIP library never
 * links, loads or calls it.
 *
 * Design (Section 2.2.1 and Section 2.2.2): Steps 1-3 and the thresholds are
 * data-parallel loops over image rows (the paper's parallel-for pattern; here
 * OpenMP instead of Cilk Plus, static row blocks), and Step 4, hysteresis,
 * stays serial, which the paper names as the main source of forced serial
 * work.  The per-pixel arithmetic is the oracle's (fp64, clamp-indexed reads,
 * separable Gaussian, Sobel, L2 strength, interpolated suppression, the same
 * operation order), so the result equals the oracle's bit for bit; the serial
 * part calls the oracle's breadth-first hysteresis.
 *
 * The two parts are timed separately so that the parallel fraction f of the
 * paper's Amdahl discussion (the asymmetric-multicore speedup formula in
 * Section 2.2.1) can be measured rather than assumed.
 */
#define _POSIX_C_SOURCE 199309L
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

long oracle_hysteresis(const uint8_t* cls, int H, int W, uint8_t* edges);
void oracle_gauss_weights(double sigma, int R, double* g);

static int cl(int v, int n) { return v < 0 ? 0 : (v > n - 1 ? n - 1 : v); }

static double now_s(void) {
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

static double sgn(double v) { return (v > 0.0) - (v < 0.0); }

/* Float Canny, Steps 1-4, relative (low/high times the largest strength) or
 * absolute thresholds.  Writes edges (255 / 0, H*W) and the seconds spent in
 * the parallel part (Steps 1-3 and the thresholds) and in the serial part
 * (hysteresis).  Returns 0, or -1 if memory runs out. */
int pd_canny_f32(const float* X, int H, int W, double sigma, int R, double low, double high,
                 int relative, int nthreads, uint8_t* edges, double* t_parallel,
                 double* t_serial) {
    const long n = (long)H * W;
    double* g = (double*)malloc((2 * R + 1) * sizeof(double));
    double* T = (double*)malloc((n > 0 ? n : 1) * sizeof(double));
    double* B = (double*)malloc((n > 0 ? n : 1) * sizeof(double));
    double* Gx = (double*)malloc((n > 0 ? n : 1) * sizeof(double));
    double* Gy = (double*)malloc((n > 0 ? n : 1) * sizeof(double));
    double* M = (double*)malloc((n > 0 ? n : 1) * sizeof(double));
    uint8_t* cls = (uint8_t*)malloc(n > 0 ? n : 1);
    if (!g || !T || !B || !Gx || !Gy || !M || !cls) {
        free(g); free(T); free(B); free(Gx); free(Gy); free(M); free(cls);
        return -1;
    }
    const double t0 = now_s();
    oracle_gauss_weights(sigma, R, g);
    /* Step 1: horizontal then vertical pass, clamped reads */
#pragma omp parallel for schedule(static) num_threads(nthreads)
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            double a = 0.0;
            for (int k = -R; k <= R; ++k) a += g[k + R] * (double)X[(long)y * W + cl(x + k, W)];
            T[(long)y * W + x] = a;
        }
#pragma omp parallel for schedule(static) num_threads(nthreads)
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            double a = 0.0;
            for (int k = -R; k <= R; ++k) a += g[k + R] * T[(long)cl(y + k, H) * W + x];
            B[(long)y * W + x] = a;
        }
    /* Step 2: Sobel pair (correlation, x right, y down) and L2 strength */
    double mx = 0.0;
#pragma omp parallel for schedule(static) num_threads(nthreads) reduction(max : mx)
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            static const double s[3] = {1.0, 2.0, 1.0};
            double gx = 0.0, gy = 0.0;
            for (int i = -1; i <= 1; ++i) {
                gx += s[i + 1] * (B[(long)cl(y + i, H) * W + cl(x + 1, W)] -
                                  B[(long)cl(y + i, H) * W + cl(x - 1, W)]);
                gy += s[i + 1] * (B[(long)cl(y + 1, H) * W + cl(x + i, W)] -
                                  B[(long)cl(y - 1, H) * W + cl(x + i, W)]);
            }
            const long k = (long)y * W + x;
            Gx[k] = gx;
            Gy[k] = gy;
            M[k] = sqrt(gx * gx + gy * gy);
            if (M[k] > mx) mx = M[k];
        }
    const double lo = relative ? low * mx : low;
    const double hi = relative ? high * mx : high;
    /* Step 3 and the double threshold: suppression against the two values
     * interpolated on the 3x3 ring along the gradient; keep iff M > back and
     * M >= forward, M = 0 never kept */
#pragma omp parallel for schedule(static) num_threads(nthreads)
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            const long k = (long)y * W + x;
            const double ax = fabs(Gx[k]), ay = fabs(Gy[k]);
            const int sx = (int)sgn(Gx[k]), sy = (int)sgn(Gy[k]);
            double mf = 0.0, mb = 0.0;
#define MAT(yy, xx) M[(long)cl((yy), H) * W + cl((xx), W)]
            if (ax >= ay && ax > 0.0) {
                const double t = ay / ax;
                const double mp = (1.0 - t) * MAT(y, x + sx) + t * MAT(y + sy, x + sx);
                const double mm = (1.0 - t) * MAT(y, x - sx) + t * MAT(y - sy, x - sx);
                if (sx > 0) { mf = mp; mb = mm; } else { mf = mm; mb = mp; }
            } else if (ay > ax) {
                const double t = ax / ay;
                const double mp = (1.0 - t) * MAT(y + sy, x) + t * MAT(y + sy, x + sx);
                const double mm = (1.0 - t) * MAT(y - sy, x) + t * MAT(y - sy, x - sx);
                if (sy > 0) { mf = mp; mb = mm; } else { mf = mm; mb = mp; }
            }
#undef MAT
            const int keep = (M[k] > 0.0) && (M[k] > mb) && (M[k] >= mf);
            cls[k] = (uint8_t)((keep && M[k] > hi) ? 2 : ((keep && M[k] >= lo) ? 1 : 0));
        }
    const double t1 = now_s();
    /* Step 4: serial hysteresis (breadth-first search from the strong pixels) */
    oracle_hysteresis(cls, H, W, edges);
    const double t2 = now_s();
    *t_parallel = t1 - t0;
    *t_serial = t2 - t1;
    free(g); free(T); free(B); free(Gx); free(Gy); free(M); free(cls);
    return 0;
}
