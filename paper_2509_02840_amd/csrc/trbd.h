// trbd.h -- truncated bidiagonal approximation of a handle's factorization
// (Section 1.3, eqs. (trBD), (errtrBD)).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bdu {

// Scratch: t (n doubles), rank (n int64).  Outputs: idx (r), err2 (1),
// Qr (m x r, leading dimension m), Pr (n x r, leading dimension n).
hipError_t launch_trbd(const double *Q, int64_t ldq, int64_t m, const double *P, int64_t ldp, int64_t n,
                       const double *d, const double *e, int64_t r, double *t, int64_t *rank, int64_t *idx,
                       double *err2, double *Qr, double *Pr, hipStream_t st);

}  // namespace bdu
