// Differentiable front end: workspace sizing and dispatch by radius to the
// radius-group translation units (canny_mag_g1..6.hip).
#include "canny_mag_impl.h"

namespace canny {

size_t mag_partials(int N, int H, int W, int radius) {
    // one partial per wave of the second backward kernel (halo (radius+3)/4 lanes)
    const int hl = (radius + 3) / 4;
    const int sc = 4 * (kWave - 2 * hl);
    return (size_t)N * ceil_div(W, sc) * ceil_div(H, kMagRows);
}

// radius -> group (groups balance compile cost, which grows about as R^2)
static int mag_group(int radius) {
    switch (radius) {
        case 12: return 1;
        case 11: return 2;
        case 10: return 3;
        case 9: case 1: case 2: return 4;
        case 8: case 3: case 4: return 5;
        case 7: case 5: case 6: return 6;
        default: return 0;
    }
}

hipError_t launch_mag_forward(const float* I, const float* sigma, int N, int H, int W, int radius,
                              float* M, hipStream_t s) {
    switch (mag_group(radius)) {
#define CASE(g) case g: return mag_forward_g##g(I, sigma, N, H, W, radius, M, s);
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6)
#undef CASE
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_mag_backward(const float* I, const float* sigma, const float* dM, int N, int H, int W,
                               int radius, float* dI, float* dsigma, float* dB, float* partial,
                               hipStream_t s) {
    switch (mag_group(radius)) {
#define CASE(g) case g: return mag_backward_g##g(I, sigma, dM, N, H, W, radius, dI, dsigma, dB, partial, s);
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6)
#undef CASE
        default: return hipErrorInvalidValue;
    }
}

}  // namespace canny
