// Differentiable front end, radius group 4 (radii 1, 2, 9): the
// unrolled kernels of canny_mag_impl.h instantiated for these radii only, so
// that the radius groups compile in parallel.
#include "canny_mag_impl.h"

namespace canny {

hipError_t mag_forward_g4(const float* I, const float* sigma, int N, int H, int W, int radius,
                           float* M, hipStream_t s) {
    switch (radius) {
#define CASE(r) case r: return fwd_r<r>(I, sigma, N, H, W, M, s);
        CASE(1) CASE(2) CASE(9)
#undef CASE
        default: return hipErrorInvalidValue;
    }
}

hipError_t mag_backward_g4(const float* I, const float* sigma, const float* dM, int N, int H, int W,
                            int radius, float* dI, float* dsigma, float* dB, float* partial,
                            hipStream_t s) {
    switch (radius) {
#define CASE(r) case r: return bwd_r<r>(I, sigma, dM, N, H, W, dI, dsigma, dB, partial, s);
        CASE(1) CASE(2) CASE(9)
#undef CASE
        default: return hipErrorInvalidValue;
    }
}

}  // namespace canny
