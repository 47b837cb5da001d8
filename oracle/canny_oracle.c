/*
 * canny_oracle.c -- plain, slow CPU oracle for the Canny edge detector.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The product path
 * (the HIP library) never links, loads or calls it, and the two share no
 * code, headers, tables or helpers.
 *
 * What it computes follows the paper's four steps (Section 2.2.1, Steps 1-4,
 * and the pipeline order of Algorithm 1):
 *   Step 1  noise filter (Gaussian; integer path: 5x5 binomial),
 *   Step 2  Sobel gradients Gx, Gy, gradient strength and direction,
 *   Step 3  non-maximum suppression,
 *   Step 4  hysteresis with a lower and an upper threshold.
 * Where the paper is silent (border rule, rounding, tie rule, connectivity,
 * magnitude norm, direction quantisation) the readings listed in the design
 * notes are used; each function states the reading it implements.
 *
 * Style: every stage is written as its plain definition, with clamp-indexed
 * reads at every stage (replicate border), full 2-D sums instead of separable
 * ones where the definition is 2-D, atan2 for the direction, breadth-first
 * search for hysteresis, and fp64 for all floating point.  No blocking, no
 * fusion, no reordering.
 *
 * Parity pins: every exported function is pinned in tests/test_oracle_pins.py
 * against closed forms, library special cases or brute force.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* replicate border: clamp an index into [0, n-1] */
static int clampi(int v, int n) {
    if (v < 0) return 0;
    if (v > n - 1) return n - 1;
    return v;
}

/* ------------------------------------------------------------------------
 * Integer path
 * ---------------------------------------------------------------------- */

/* Step 1 (Section 2.2.1), integer form: 5x5 binomial filter with weights
 * b = (1,4,6,4,1) in each axis, i.e. the 2-D sum S = sum_i sum_j b_i b_j
 * I(cy(y+i), cx(x+j)), rounded once, half up: B = (S + 128) >> 8. */
void oracle_blur_binomial(const uint8_t* I, int H, int W, uint8_t* B) {
    static const int b[5] = {1, 4, 6, 4, 1};
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            long S = 0;
            for (int i = -2; i <= 2; ++i)
                for (int j = -2; j <= 2; ++j)
                    S += (long)b[i + 2] * b[j + 2] *
                         I[(long)clampi(y + i, H) * W + clampi(x + j, W)];
            B[(long)y * W + x] = (uint8_t)((S + 128) >> 8);
        }
    }
}

/* Step 2 (Section 2.2.1): the Sobel mask pair as a correlation, x to the
 * right and y downwards, on the clamped (replicate-border) blurred image:
 *   Gx = sum_i s_i [B(y+i, x+1) - B(y+i, x-1)],
 *   Gy = sum_j s_j [B(y+1, x+j) - B(y-1, x+j)],  s = (1,2,1). */
void oracle_sobel_i32(const uint8_t* B, int H, int W, int32_t* Gx, int32_t* Gy) {
    static const int s[3] = {1, 2, 1};
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            int gx = 0, gy = 0;
            for (int i = -1; i <= 1; ++i) {
                gx += s[i + 1] * ((int)B[(long)clampi(y + i, H) * W + clampi(x + 1, W)] -
                                  (int)B[(long)clampi(y + i, H) * W + clampi(x - 1, W)]);
                gy += s[i + 1] * ((int)B[(long)clampi(y + 1, H) * W + clampi(x + i, W)] -
                                  (int)B[(long)clampi(y - 1, H) * W + clampi(x + i, W)]);
            }
            Gx[(long)y * W + x] = gx;
            Gy[(long)y * W + x] = gy;
        }
    }
}

/* Gradient direction (Algorithm 1 computes theta from the two gradient
 * components; read as the gradient angle atan2(Gy, Gx) modulo 180 degrees),
 * quantised to the nearest multiple of 45 degrees.  Codes:
 *   0 = horizontal neighbours (0 deg),  1 = diagonal (+1,+1) (45 deg),
 *   2 = vertical neighbours (90 deg),   3 = anti-diagonal (+1,-1) (135 deg).
 * With y pointing down, 45 deg is the (dy,dx) = (1,1) diagonal. */
int oracle_sector(int gx, int gy) {
    double th = atan2((double)gy, (double)gx) * (180.0 / M_PI); /* (-180, 180] */
    if (th < 0.0) th += 180.0;                                  /* [0, 180]    */
    int q = (int)floor(th / 45.0 + 0.5);
    return q & 3; /* 180 deg folds onto 0 */
}

void oracle_sector_array(const int32_t* gx, const int32_t* gy, long n, uint8_t* out) {
    for (long k = 0; k < n; ++k) out[k] = (uint8_t)oracle_sector(gx[k], gy[k]);
}

/* neighbour step d = (dy, dx) along each quantised direction */
static const int kSecDy[4] = {0, 1, 1, 1};
static const int kSecDx[4] = {1, 1, 0, -1};

/* Steps 1-3 plus the double threshold of Step 4, integer path.
 *   M = |Gx| + |Gy| (gradient strength, L1 norm),
 *   NMS keeps p iff M(p) > M(p-d) and M(p) >= M(p+d) with clamped neighbours
 *   (ties go to the earlier pixel in raster order),
 *   class 2 (strong) iff kept and M > high, class 1 (weak) iff kept and
 *   low <= M <= high, else 0.
 * Optional outputs M_out (int32 H*W) and sec_out (uint8 H*W) may be NULL. */
void oracle_classify_u8(const uint8_t* I, int H, int W, int low, int high, uint8_t* cls,
                        int32_t* M_out, uint8_t* sec_out) {
    long n = (long)H * W;
    uint8_t* B = (uint8_t*)malloc(n);
    int32_t* Gx = (int32_t*)malloc(n * sizeof(int32_t));
    int32_t* Gy = (int32_t*)malloc(n * sizeof(int32_t));
    int32_t* M = (int32_t*)malloc(n * sizeof(int32_t));
    oracle_blur_binomial(I, H, W, B);
    oracle_sobel_i32(B, H, W, Gx, Gy);
    for (long k = 0; k < n; ++k) M[k] = abs(Gx[k]) + abs(Gy[k]);
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            long k = (long)y * W + x;
            int sec = oracle_sector(Gx[k], Gy[k]);
            int dy = kSecDy[sec], dx = kSecDx[sec];
            int mb = M[(long)clampi(y - dy, H) * W + clampi(x - dx, W)];
            int mf = M[(long)clampi(y + dy, H) * W + clampi(x + dx, W)];
            int keep = (M[k] > mb) && (M[k] >= mf);
            uint8_t c = 0;
            if (keep && M[k] > high) c = 2;
            else if (keep && M[k] >= low) c = 1;
            cls[k] = c;
            if (sec_out) sec_out[k] = (uint8_t)sec;
        }
    }
    if (M_out) memcpy(M_out, M, n * sizeof(int32_t));
    free(B); free(Gx); free(Gy); free(M);
}

/* Step 4 (Section 2.2.1), hysteresis: a pixel above the upper threshold is
 * an edge; a pixel between the thresholds is an edge only if it is connected
 * to one above the upper threshold.  Connectivity: 8-neighbour paths through
 * candidate pixels (class >= 1).  Breadth-first search from every strong
 * pixel.  Output 255 on edges, 0 elsewhere.  Returns the number of BFS
 * levels of the deepest search (0 if there is no strong pixel). */
long oracle_hysteresis(const uint8_t* cls, int H, int W, uint8_t* edges) {
    long n = (long)H * W;
    int32_t* queue = (int32_t*)malloc((n > 0 ? n : 1) * sizeof(int32_t));
    int32_t* depth = (int32_t*)malloc((n > 0 ? n : 1) * sizeof(int32_t));
    long head = 0, tail = 0, maxdepth = 0;
    memset(edges, 0, n);
    for (long k = 0; k < n; ++k) {
        if (cls[k] == 2) {
            edges[k] = 255;
            depth[k] = 1;
            queue[tail++] = (int32_t)k;
        }
    }
    while (head < tail) {
        long k = queue[head++];
        int y = (int)(k / W), x = (int)(k % W);
        if (depth[k] > maxdepth) maxdepth = depth[k];
        for (int dy = -1; dy <= 1; ++dy) {
            for (int dx = -1; dx <= 1; ++dx) {
                int yy = y + dy, xx = x + dx;
                if (yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
                long q = (long)yy * W + xx;
                if (cls[q] >= 1 && edges[q] == 0) {
                    edges[q] = 255;
                    depth[q] = depth[k] + 1;
                    queue[tail++] = (int32_t)q;
                }
            }
        }
    }
    free(queue);
    free(depth);
    return maxdepth;
}

/* Whole integer pipeline: Steps 1-4.  cls may be NULL. */
void oracle_canny_u8(const uint8_t* I, int H, int W, int low, int high, uint8_t* edges,
                     uint8_t* cls) {
    long n = (long)H * W;
    uint8_t* c = cls ? cls : (uint8_t*)malloc(n > 0 ? n : 1);
    oracle_classify_u8(I, H, W, low, high, c, NULL, NULL);
    oracle_hysteresis(c, H, W, edges);
    if (!cls) free(c);
}

/* ------------------------------------------------------------------------
 * Floating-point path (fp64 throughout)
 * ---------------------------------------------------------------------- */

/* Step 1, Gaussian form: taps k = -R..R sampled from exp(-k^2 / (2 sigma^2))
 * and normalised to sum 1.  g has 2R+1 entries, g[k+R] is tap k. */
void oracle_gauss_weights(double sigma, int R, double* g) {
    double s = 0.0;
    for (int k = -R; k <= R; ++k) {
        g[k + R] = exp(-(double)k * k / (2.0 * sigma * sigma));
        s += g[k + R];
    }
    for (int k = -R; k <= R; ++k) g[k + R] /= s;
}

/* d g_k / d sigma for the normalised sampled Gaussian above. */
void oracle_gauss_weights_dsigma(double sigma, int R, double* dg) {
    double* g = (double*)malloc((2 * R + 1) * sizeof(double));
    oracle_gauss_weights(sigma, R, g);
    double m2 = 0.0;
    for (int k = -R; k <= R; ++k) m2 += g[k + R] * k * k;
    for (int k = -R; k <= R; ++k)
        dg[k + R] = g[k + R] * ((double)k * k - m2) / (sigma * sigma * sigma);
    free(g);
}

/* separable clamped filtering: T = horizontal pass, out = vertical pass */
static void filter_h(const double* X, int H, int W, const double* g, int R, double* T) {
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            double a = 0.0;
            for (int k = -R; k <= R; ++k) a += g[k + R] * X[(long)y * W + clampi(x + k, W)];
            T[(long)y * W + x] = a;
        }
}
static void filter_v(const double* T, int H, int W, const double* g, int R, double* out) {
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            double a = 0.0;
            for (int k = -R; k <= R; ++k) a += g[k + R] * T[(long)clampi(y + k, H) * W + x];
            out[(long)y * W + x] = a;
        }
}

/* Step 1, float: B = sum_k g_k sum_j g_j X(cy(y+k), cx(x+j)), computed as a
 * clamped horizontal pass then a clamped vertical pass (per-axis clamping of
 * a separable kernel equals 2-D clamping). */
void oracle_gauss_blur(const double* X, int H, int W, double sigma, int R, double* B) {
    long n = (long)H * W;
    double* g = (double*)malloc((2 * R + 1) * sizeof(double));
    double* T = (double*)malloc((n > 0 ? n : 1) * sizeof(double));
    oracle_gauss_weights(sigma, R, g);
    filter_h(X, H, W, g, R, T);
    filter_v(T, H, W, g, R, B);
    free(g); free(T);
}

/* Step 2, float: Sobel pair on the clamped blurred image (same orientation
 * as the integer path). */
void oracle_sobel_f64(const double* B, int H, int W, double* Gx, double* Gy) {
    static const double s[3] = {1.0, 2.0, 1.0};
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            double gx = 0.0, gy = 0.0;
            for (int i = -1; i <= 1; ++i) {
                gx += s[i + 1] * (B[(long)clampi(y + i, H) * W + clampi(x + 1, W)] -
                                  B[(long)clampi(y + i, H) * W + clampi(x - 1, W)]);
                gy += s[i + 1] * (B[(long)clampi(y + 1, H) * W + clampi(x + i, W)] -
                                  B[(long)clampi(y - 1, H) * W + clampi(x + i, W)]);
            }
            Gx[(long)y * W + x] = gx;
            Gy[(long)y * W + x] = gy;
        }
}

static double sgn(double v) { return (v > 0.0) - (v < 0.0); }
static double Mat(const double* M, int H, int W, int y, int x) {
    return M[(long)clampi(y, H) * W + clampi(x, W)];
}

/* Steps 1-3 and the double threshold of Step 4, floating-point path.
 * X is the fp32 input image (row-major, H*W).  Gradient strength is the L2
 * norm M = sqrt(Gx^2 + Gy^2).  Non-maximum suppression uses the continuous
 * gradient direction: the two values compared against M(p) are interpolated
 * linearly on the ring of the 3x3 neighbourhood, where the gradient line
 * through p leaves it:
 *   |Gx| >= |Gy|, t = |Gy|/|Gx|:  M+ = (1-t) M(y, x+sx) + t M(y+sy, x+sx),
 *                                 M- = (1-t) M(y, x-sx) + t M(y-sy, x-sx);
 *   |Gy| >  |Gx|, t = |Gx|/|Gy|:  M+ = (1-t) M(y+sy, x) + t M(y+sy, x+sx),
 *                                 M- = (1-t) M(y-sy, x) + t M(y-sy, x-sx),
 * with sx, sy the signs of Gx, Gy and clamped reads.  "Forward" is the side
 * whose step along the dominant axis is positive; keep iff M > M(back) and
 * M >= M(forward) (same raster tie rule as the integer path); M = 0 is never
 * kept.  If relative != 0, thresholds are low*mx and high*mx with mx the
 * largest M over the image (before suppression).  Outputs:
 *   cls  uint8 H*W class map (0 none, 1 weak, 2 strong),
 *   M    double H*W magnitudes (may be NULL),
 *   amb  uint8 H*W "ambiguous" bit flags (may be NULL), set where a decision
 *        is within tol of flipping:
 *          bit 0: |M-low| <= tol*low or |M-high| <= tol*high (threshold),
 *          bit 1: M > 0 and |M - M(back)| <= tol*M or |M - M(fwd)| <= tol*M
 *                 (suppression near-tie),
 *          bit 2: min(|Gx|,|Gy|) <= tol*M or ||Gx|-|Gy|| <= tol*M
 *                 (direction within tol of a 45-degree sector boundary),
 *   mx_out  the maximum magnitude (may be NULL).
 * Returns the number of pixels with bit 0 or bit 1 set. */
long oracle_classify_f32(const float* X, int H, int W, double sigma, int R, double low,
                         double high, int relative, double tol, uint8_t* cls, double* M_out,
                         uint8_t* amb, double* mx_out) {
    long n = (long)H * W;
    double* Xd = (double*)malloc(n * sizeof(double));
    double* B = (double*)malloc(n * sizeof(double));
    double* Gx = (double*)malloc(n * sizeof(double));
    double* Gy = (double*)malloc(n * sizeof(double));
    double* M = (double*)malloc(n * sizeof(double));
    for (long k = 0; k < n; ++k) Xd[k] = (double)X[k];
    oracle_gauss_blur(Xd, H, W, sigma, R, B);
    oracle_sobel_f64(B, H, W, Gx, Gy);
    double mx = 0.0;
    for (long k = 0; k < n; ++k) {
        M[k] = sqrt(Gx[k] * Gx[k] + Gy[k] * Gy[k]);
        if (M[k] > mx) mx = M[k];
    }
    double lo = relative ? low * mx : low;
    double hi = relative ? high * mx : high;
    long namb = 0;
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            long k = (long)y * W + x;
            double ax = fabs(Gx[k]), ay = fabs(Gy[k]);
            double sx = sgn(Gx[k]), sy = sgn(Gy[k]);
            double mf, mb; /* forward / backward interpolated magnitudes */
            if (ax >= ay && ax > 0.0) {
                double t = ay / ax;
                double mp = (1.0 - t) * Mat(M, H, W, y, x + (int)sx) +
                            t * Mat(M, H, W, y + (int)sy, x + (int)sx);
                double mm = (1.0 - t) * Mat(M, H, W, y, x - (int)sx) +
                            t * Mat(M, H, W, y - (int)sy, x - (int)sx);
                /* dominant axis x: forward is the side at x+1 */
                if (sx > 0) { mf = mp; mb = mm; } else { mf = mm; mb = mp; }
            } else if (ay > ax) {
                double t = ax / ay;
                double mp = (1.0 - t) * Mat(M, H, W, y + (int)sy, x) +
                            t * Mat(M, H, W, y + (int)sy, x + (int)sx);
                double mm = (1.0 - t) * Mat(M, H, W, y - (int)sy, x) +
                            t * Mat(M, H, W, y - (int)sy, x - (int)sx);
                /* dominant axis y: forward is the side at y+1 */
                if (sy > 0) { mf = mp; mb = mm; } else { mf = mm; mb = mp; }
            } else {
                mf = mb = 0.0; /* M == 0 */
            }
            int keep = (M[k] > 0.0) && (M[k] > mb) && (M[k] >= mf);
            uint8_t c = 0;
            if (keep && M[k] > hi) c = 2;
            else if (keep && M[k] >= lo) c = 1;
            cls[k] = c;
            if (amb) {
                double m = M[k];
                int a = 0;
                if (fabs(m - lo) <= tol * lo || fabs(m - hi) <= tol * hi) a |= 1;
                if (m > 0.0 && (fabs(m - mb) <= tol * m || fabs(m - mf) <= tol * m)) a |= 2;
                if (fmin(ax, ay) <= tol * m || fabs(ax - ay) <= tol * m) a |= 4;
                amb[k] = (uint8_t)a;
                namb += (a & 3) != 0;
            }
        }
    }
    if (M_out) memcpy(M_out, M, n * sizeof(double));
    if (mx_out) *mx_out = mx;
    free(Xd); free(B); free(Gx); free(Gy); free(M);
    return namb;
}

/* Gradient direction of the float path quantised to four sectors, as in
 * the integer path (the nearest multiple of 45 degrees of atan2(Gy, Gx)
 * modulo 180; Algorithm 1 forms an explicit direction angle), codes as in
 * oracle_sector.  Used by the four-sector variant below. */
int oracle_sector_f64(double gx, double gy) {
    double th = atan2(gy, gx) * (180.0 / M_PI);
    if (th < 0.0) th += 180.0;
    int q = (int)floor(th / 45.0 + 0.5);
    return q & 3;
}

/* Steps 1-3 and the double threshold, float path with the four-sector
 * direction: Gaussian, Sobel and L2 strength exactly as in
 * oracle_classify_f32, then suppression against the two 8-neighbours
 * p - d and p + d along the quantised direction d (clamped reads): keep iff
 * M > 0, M > M(p - d) and M >= M(p + d) (the raster tie rule of the integer
 * path).  Thresholds as in oracle_classify_f32.  amb bit flags:
 *   bit 0: within tol of a threshold, bit 1: suppression near-tie,
 *   bit 3: direction near a sector boundary, |ay - k ax| <= 4 tol M for
 *          k = tan(22.5 deg) or tan(67.5 deg) (an fp32 evaluation of the
 *          boundary test can land on either side there), or M = 0.
 * Returns the number of pixels with bit 0, 1 or 3 set. */
long oracle_classify_f32_sector(const float* X, int H, int W, double sigma, int R, double low,
                                double high, int relative, double tol, uint8_t* cls,
                                double* M_out, uint8_t* amb, double* mx_out) {
    long n = (long)H * W;
    double* Xd = (double*)malloc(n * sizeof(double));
    double* B = (double*)malloc(n * sizeof(double));
    double* Gx = (double*)malloc(n * sizeof(double));
    double* Gy = (double*)malloc(n * sizeof(double));
    double* M = (double*)malloc(n * sizeof(double));
    for (long k = 0; k < n; ++k) Xd[k] = (double)X[k];
    oracle_gauss_blur(Xd, H, W, sigma, R, B);
    oracle_sobel_f64(B, H, W, Gx, Gy);
    double mx = 0.0;
    for (long k = 0; k < n; ++k) {
        M[k] = sqrt(Gx[k] * Gx[k] + Gy[k] * Gy[k]);
        if (M[k] > mx) mx = M[k];
    }
    double lo = relative ? low * mx : low;
    double hi = relative ? high * mx : high;
    const double k1 = sqrt(2.0) - 1.0, k2 = sqrt(2.0) + 1.0;
    long namb = 0;
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            long k = (long)y * W + x;
            int sec = oracle_sector_f64(Gx[k], Gy[k]);
            int dy = kSecDy[sec], dx = kSecDx[sec];
            double mb = Mat(M, H, W, y - dy, x - dx);
            double mf = Mat(M, H, W, y + dy, x + dx);
            int keep = (M[k] > 0.0) && (M[k] > mb) && (M[k] >= mf);
            uint8_t c = 0;
            if (keep && M[k] > hi) c = 2;
            else if (keep && M[k] >= lo) c = 1;
            cls[k] = c;
            if (amb) {
                double m = M[k], ax = fabs(Gx[k]), ay = fabs(Gy[k]);
                int a = 0;
                if (fabs(m - lo) <= tol * lo || fabs(m - hi) <= tol * hi) a |= 1;
                if (m > 0.0 && (fabs(m - mb) <= tol * m || fabs(m - mf) <= tol * m)) a |= 2;
                if (m == 0.0 || fabs(ay - k1 * ax) <= 4.0 * tol * m || fabs(ay - k2 * ax) <= 4.0 * tol * m)
                    a |= 8;
                amb[k] = (uint8_t)a;
                namb += (a & 11) != 0;
            }
        }
    }
    if (M_out) memcpy(M_out, M, n * sizeof(double));
    if (mx_out) *mx_out = mx;
    free(Xd); free(B); free(Gx); free(Gy); free(M);
    return namb;
}

/* ------------------------------------------------------------------------
 * Differentiable front end M(I, sigma) = |Sobel * G_sigma * I| (L2 norm)
 * ---------------------------------------------------------------------- */

/* Forward: M for one image at scale sigma with fixed radius R. */
void oracle_mag_forward(const double* I, int H, int W, double sigma, int R, double* M) {
    long n = (long)H * W;
    double* B = (double*)malloc(n * sizeof(double));
    double* Gx = (double*)malloc(n * sizeof(double));
    double* Gy = (double*)malloc(n * sizeof(double));
    oracle_gauss_blur(I, H, W, sigma, R, B);
    oracle_sobel_f64(B, H, W, Gx, Gy);
    for (long k = 0; k < n; ++k) M[k] = sqrt(Gx[k] * Gx[k] + Gy[k] * Gy[k]);
    free(B); free(Gx); free(Gy);
}

/* Backward of the forward above, given gM = dL/dM.  Each forward stage is
 * transposed literally: every clamped read in the forward becomes a
 * scatter-add onto the clamped pixel.  dM/dG = G/M, taken as 0 where M = 0.
 *   dI       = G_h^T G_v^T (Sobel_x^T (gM Gx/M) + Sobel_y^T (gM Gy/M)),
 *   dsigma   = sum_p dB(p) * dB(p)/dsigma, with
 *              dB/dsigma = G_v'(G_h I) + G_v(G_h' I), G' the tap derivatives.
 * dI is H*W; *dsigma receives one scalar. */
void oracle_mag_backward(const double* I, int H, int W, double sigma, int R, const double* gM,
                         double* dI, double* dsigma) {
    long n = (long)H * W;
    int nt = 2 * R + 1;
    double* g = (double*)malloc(nt * sizeof(double));
    double* dg = (double*)malloc(nt * sizeof(double));
    double* T = (double*)malloc(n * sizeof(double));
    double* B = (double*)malloc(n * sizeof(double));
    double* Gx = (double*)malloc(n * sizeof(double));
    double* Gy = (double*)malloc(n * sizeof(double));
    double* dB = (double*)calloc(n, sizeof(double));
    double* dT = (double*)calloc(n, sizeof(double));
    double* Tp = (double*)malloc(n * sizeof(double));
    double* Bs = (double*)malloc(n * sizeof(double));
    double* tmp = (double*)malloc(n * sizeof(double));
    static const double s[3] = {1.0, 2.0, 1.0};
    oracle_gauss_weights(sigma, R, g);
    oracle_gauss_weights_dsigma(sigma, R, dg);
    filter_h(I, H, W, g, R, T);
    filter_v(T, H, W, g, R, B);
    oracle_sobel_f64(B, H, W, Gx, Gy);
    /* Sobel^T: scatter dGx, dGy back onto the clamped taps */
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            long k = (long)y * W + x;
            double m = sqrt(Gx[k] * Gx[k] + Gy[k] * Gy[k]);
            double dgx = m > 0.0 ? gM[k] * Gx[k] / m : 0.0;
            double dgy = m > 0.0 ? gM[k] * Gy[k] / m : 0.0;
            for (int i = -1; i <= 1; ++i) {
                dB[(long)clampi(y + i, H) * W + clampi(x + 1, W)] += s[i + 1] * dgx;
                dB[(long)clampi(y + i, H) * W + clampi(x - 1, W)] -= s[i + 1] * dgx;
                dB[(long)clampi(y + 1, H) * W + clampi(x + i, W)] += s[i + 1] * dgy;
                dB[(long)clampi(y - 1, H) * W + clampi(x + i, W)] -= s[i + 1] * dgy;
            }
        }
    /* G_v^T then G_h^T */
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x)
            for (int k = -R; k <= R; ++k)
                dT[(long)clampi(y + k, H) * W + x] += g[k + R] * dB[(long)y * W + x];
    memset(dI, 0, n * sizeof(double));
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x)
            for (int k = -R; k <= R; ++k)
                dI[(long)y * W + clampi(x + k, W)] += g[k + R] * dT[(long)y * W + x];
    /* dB/dsigma = G_v'(T) + G_v(G_h' I) */
    filter_h(I, H, W, dg, R, Tp);
    filter_v(T, H, W, dg, R, Bs);
    filter_v(Tp, H, W, g, R, tmp);
    double acc = 0.0;
    for (long k = 0; k < n; ++k) acc += dB[k] * (Bs[k] + tmp[k]);
    *dsigma = acc;
    free(g); free(dg); free(T); free(B); free(Gx); free(Gy); free(dB); free(dT);
    free(Tp); free(Bs); free(tmp);
}

/* ------------------------------------------------------------------------
 * Laplacian zero-crossing detector (the comparator the paper's introduction
 * sets Canny against, Laplace(f) = f_xx + f_yy), integer path
 * ---------------------------------------------------------------------- */

/* The Laplace operator on the Step-1-filtered image B (the same 5x5 binomial
 * as the integer Canny path), as the sum of the second central differences
 * along each axis, with clamped (replicate-border) reads:
 *   L(y,x) = [B(y,x-1) - 2 B(y,x) + B(y,x+1)] + [B(y-1,x) - 2 B(y,x) + B(y+1,x)]. */
void oracle_laplace_i32(const uint8_t* B, int H, int W, int32_t* L) {
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            int c = B[(long)y * W + x];
            int dxx = (int)B[(long)y * W + clampi(x - 1, W)] - 2 * c + (int)B[(long)y * W + clampi(x + 1, W)];
            int dyy = (int)B[(long)clampi(y - 1, H) * W + x] - 2 * c + (int)B[(long)clampi(y + 1, H) * W + x];
            L[(long)y * W + x] = dxx + dyy;
        }
    }
}

/* Zero crossings of L, two cases.
 *  (a) Between two pixels: every pair of 4-neighbours (p, q), q the right or
 *      the lower neighbour of p, both inside the image, is visited once; the
 *      pair crosses iff L(p) and L(q) have strictly opposite signs (one > 0,
 *      the other < 0) and |L(p) - L(q)| >= t.  The crossing is marked on the
 *      one whose |L| is smaller (the one nearer the zero), on p when they are
 *      equal (the earlier pixel in raster order).
 *  (b) At a pixel: p with L(p) = 0 is marked iff its left and right
 *      neighbours, or its upper and lower neighbours (all inside the image),
 *      have strictly opposite signs with |difference| >= t.
 * Zeros never cross in (a), so a Laplacian that returns to 0 (the tail of a
 * blurred step) marks nothing; a zero run of two or more pixels between
 * opposite signs marks nothing either.
 * edges: 255 on marked pixels, 0 elsewhere.  Returns the number of marked
 * pixels. */
static int strictly_opposite(int a, int b) { return (a > 0 && b < 0) || (a < 0 && b > 0); }

long oracle_zero_crossings(const int32_t* L, int H, int W, int t, uint8_t* edges) {
    long n = (long)H * W, count = 0;
    memset(edges, 0, n);
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            long p = (long)y * W + x;
            /* (a) the pairs (p, right) and (p, below) */
            for (int dir = 0; dir < 2; ++dir) {
                int yy = y + (dir == 1), xx = x + (dir == 0);
                if (yy >= H || xx >= W) continue;
                long q = (long)yy * W + xx;
                int lp = L[p], lq = L[q];
                if (!strictly_opposite(lp, lq) || abs(lp - lq) < t) continue;
                edges[abs(lp) <= abs(lq) ? p : q] = 255;
            }
            /* (b) a zero between strictly opposite neighbours */
            if (L[p] == 0) {
                if (x >= 1 && x + 1 < W) {
                    int a = L[p - 1], b = L[p + 1];
                    if (strictly_opposite(a, b) && abs(a - b) >= t) edges[p] = 255;
                }
                if (y >= 1 && y + 1 < H) {
                    int a = L[p - W], b = L[p + W];
                    if (strictly_opposite(a, b) && abs(a - b) >= t) edges[p] = 255;
                }
            }
        }
    }
    for (long k = 0; k < n; ++k) count += edges[k] != 0;
    return count;
}

/* The whole detector: B = Step 1 (5x5 binomial, one rounding), L = Laplace(B),
 * edges = zero crossings of L with slope threshold t.  L_out may be NULL. */
long oracle_log_u8(const uint8_t* I, int H, int W, int t, uint8_t* edges, int32_t* L_out) {
    long n = (long)H * W;
    uint8_t* B = (uint8_t*)malloc(n > 0 ? n : 1);
    int32_t* L = (int32_t*)malloc((n > 0 ? n : 1) * sizeof(int32_t));
    oracle_blur_binomial(I, H, W, B);
    oracle_laplace_i32(B, H, W, L);
    long count = oracle_zero_crossings(L, H, W, t, edges);
    if (L_out) memcpy(L_out, L, n * sizeof(int32_t));
    free(B);
    free(L);
    return count;
}
