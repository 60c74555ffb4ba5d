// orth.h -- orthogonality monitor and correction of the factors Q and P:
// E = X^T X - I (FP64 matrix cores), ||E||_F, and one Newton-Schulz step
// X <- X - X E / 2 towards the orthogonal polar factor of X.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bdu {

// X: ld x k column-major (ld a multiple of 128; rows past the matrix are
// zero), E: k x k in a lde x lde buffer (lde = k rounded up to 64).
hipError_t launch_orth_gram(const double *X, int64_t ld, int64_t k, double *E, int64_t lde, hipStream_t st);
// out[0] = ||E||_F (k x k part); part: lde doubles of scratch.
hipError_t launch_orth_norm(const double *E, int64_t k, int64_t lde, double *part, double *out, hipStream_t st);
// Y = X - (X E) / 2 (Y: ld x k, leading dimension ld).
hipError_t launch_orth_update(const double *X, int64_t ld, int64_t k, const double *E, int64_t lde, double *Y,
                              hipStream_t st);

}  // namespace bdu
