/*
 * sanitize_main.c -- drives every function of the CPU oracle and of the
 * paper-design baseline over small and degenerate shapes (1x1 up to a few
 * dozen pixels, radii 1-12, thresholds at and past the extremes), for a
 * build with AddressSanitizer and UndefinedBehaviorSanitizer.  Test
 * infrastructure only; the oracle's test suite compiles and runs it on the
 * CPU.  It checks nothing itself: a sanitizer report, or a non-zero exit,
 * is the failure.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void oracle_blur_binomial(const uint8_t* I, int H, int W, uint8_t* B);
void oracle_sobel_i32(const uint8_t* B, int H, int W, int32_t* Gx, int32_t* Gy);
int oracle_sector(int gx, int gy);
void oracle_sector_array(const int32_t* gx, const int32_t* gy, long n, uint8_t* out);
void oracle_classify_u8(const uint8_t* I, int H, int W, int low, int high, uint8_t* cls,
                        int32_t* M_out, uint8_t* sec_out);
long oracle_hysteresis(const uint8_t* cls, int H, int W, uint8_t* edges);
void oracle_canny_u8(const uint8_t* I, int H, int W, int low, int high, uint8_t* edges, uint8_t* cls);
void oracle_gauss_weights(double sigma, int R, double* g);
void oracle_gauss_weights_dsigma(double sigma, int R, double* dg);
void oracle_gauss_blur(const double* X, int H, int W, double sigma, int R, double* B);
void oracle_sobel_f64(const double* B, int H, int W, double* Gx, double* Gy);
long oracle_classify_f32(const float* X, int H, int W, double sigma, int R, double low,
                         double high, int relative, double tol, uint8_t* cls, double* M_out,
                         uint8_t* amb, double* mx_out);
int oracle_sector_f64(double gx, double gy);
long oracle_classify_f32_sector(const float* X, int H, int W, double sigma, int R, double low,
                                double high, int relative, double tol, uint8_t* cls,
                                double* M_out, uint8_t* amb, double* mx_out);
void oracle_mag_forward(const double* I, int H, int W, double sigma, int R, double* M);
void oracle_mag_backward(const double* I, int H, int W, double sigma, int R, const double* gM,
                         double* dI, double* dsigma);
void oracle_laplace_i32(const uint8_t* B, int H, int W, int32_t* L);
long oracle_zero_crossings(const int32_t* L, int H, int W, int t, uint8_t* edges);
long oracle_log_u8(const uint8_t* I, int H, int W, int t, uint8_t* edges, int32_t* L_out);
int pd_canny_f32(const float* X, int H, int W, double sigma, int R, double low, double high,
                 int relative, int nthreads, uint8_t* edges, double* t_parallel, double* t_serial);

static uint32_t state = 12345u;
static uint32_t next(void) {  /* xorshift32: inputs only */
    state ^= state << 13;
    state ^= state >> 17;
    state ^= state << 5;
    return state;
}

static void run(int H, int W) {
    const long n = (long)H * W;
    /* exact-size buffers, so that any read or write past n is reported */
    uint8_t* I = malloc(n);
    uint8_t* B = malloc(n);
    uint8_t* c = malloc(n);
    uint8_t* e = malloc(n);
    uint8_t* s = malloc(n);
    int32_t* gx = malloc(n * sizeof(int32_t));
    int32_t* gy = malloc(n * sizeof(int32_t));
    int32_t* M = malloc(n * sizeof(int32_t));
    float* X = malloc(n * sizeof(float));
    double* D = malloc(n * sizeof(double));
    double* D2 = malloc(n * sizeof(double));
    double* D3 = malloc(n * sizeof(double));
    double* gM = malloc(n * sizeof(double));
    for (long k = 0; k < n; ++k) {
        I[k] = (uint8_t)(next() & 255u);
        X[k] = (float)I[k];
        D[k] = I[k] / 255.0;
        gM[k] = (double)(int)(next() % 7u) - 3.0;
    }
    oracle_blur_binomial(I, H, W, B);
    oracle_sobel_i32(B, H, W, gx, gy);
    oracle_sector_array(gx, gy, n, s);
    const int lh[][2] = {{0, 0}, {40, 100}, {2040, 2040}, {5000, 6000}};
    for (int k = 0; k < 4; ++k) {
        oracle_classify_u8(I, H, W, lh[k][0], lh[k][1], c, M, s);
        oracle_hysteresis(c, H, W, e);
        oracle_canny_u8(I, H, W, lh[k][0], lh[k][1], e, NULL);
    }
    double mx = 0.0, dsig = 0.0, tp = 0.0, ts = 0.0;
    for (int R = 1; R <= 12; R += (R < 3 ? 1 : 3)) {
        double g[25], dg[25];
        oracle_gauss_weights(0.4 + 0.3 * R, R, g);
        oracle_gauss_weights_dsigma(0.4 + 0.3 * R, R, dg);
        oracle_gauss_blur(D, H, W, 0.4 + 0.3 * R, R, D2);
        oracle_sobel_f64(D2, H, W, D2, D3);
        if (R <= 8) {
            oracle_classify_f32(X, H, W, 1.4, R, 0.05, 0.15, 1, 1e-5, c, D2, s, &mx);
            oracle_classify_f32(X, H, W, 1.4, R, 10.0, 30.0, 0, 1e-5, c, NULL, NULL, NULL);
            oracle_classify_f32_sector(X, H, W, 1.4, R, 10.0, 30.0, 0, 1e-5, c, D2, s, &mx);
            if (pd_canny_f32(X, H, W, 1.4, R, 0.05, 0.15, 1, 2, e, &tp, &ts) != 0) exit(3);
        }
        oracle_mag_forward(D, H, W, 0.5 + 0.2 * R, R, D2);
        oracle_mag_backward(D, H, W, 0.5 + 0.2 * R, R, gM, D3, &dsig);
    }
    for (int t = 0; t <= 2041; t += 680) oracle_log_u8(I, H, W, t, e, M);
    oracle_laplace_i32(B, H, W, M);
    oracle_zero_crossings(M, H, W, 1, e);
    free(I); free(B); free(c); free(e); free(s); free(gx); free(gy); free(M);
    free(X); free(D); free(D2); free(D3); free(gM);
}

int main(void) {
    static const int sizes[][2] = {{1, 1}, {1, 2}, {2, 1}, {1, 7}, {7, 1}, {2, 2}, {3, 3},
                                   {3, 5}, {5, 3}, {8, 9}, {13, 31}, {33, 17}, {40, 41}};
    for (unsigned k = 0; k < sizeof(sizes) / sizeof(sizes[0]); ++k) run(sizes[k][0], sizes[k][1]);
    for (int gx = -1020; gx <= 1020; gx += 17)
        for (int gy = -1020; gy <= 1020; gy += 13) (void)(oracle_sector(gx, gy) + oracle_sector_f64(gx, gy));
    puts("sanitized oracle run: ok");
    return 0;
}
