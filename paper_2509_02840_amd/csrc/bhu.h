// bhu.h -- kernels of the Householder bidiagonal update (Section 3.3,
// Theorem 1, Algorithm 1): matrix-vector products with the reflector
// collections Y, W and the inverses S = T^{-1}, Rv = R^{-1} of eq. (TR), the
// reflector construction, and the FP64 matrix-core product that applies
// Q_k = I - 2 Y S Y^T and P_k = I - 2 W Rv W^T (eq. QP) to Q and P.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bdu {

// out[c] = alpha * sum_{r < rows} X[r + c ld] v[r] for c < cols (one
// workgroup per column, a fixed reduction tree).  cols == 0 launches nothing.
hipError_t launch_bhu_gemv_t(const double *X, int64_t ld, int64_t rows, int64_t cols, const double *v, double alpha,
                             double *out, hipStream_t st);

// out[r] = base[r] + [r == unit] + alpha * sum_{c < cols} X[r + c ld] h[c hs]
// for r < rows (base may be null: 0), through the chunk partials part
// (ceil(cols / 128) columns of lp >= rows doubles; chunks added in order).
// rows == 0 launches nothing; out may be a column of X at or beyond cols.
hipError_t launch_bhu_gemv_n(const double *X, int64_t ld, int64_t rows, int64_t cols, const double *h, int64_t hs,
                             double alpha, const double *base, int64_t unit, double *out, double *part, int64_t lp,
                             hipStream_t st);

// x = B p + bv * dot[0] (B the m x n upper bidiagonal d, e; x of length m).
hipError_t launch_bhu_bmul(const double *d, const double *e, int64_t m, int64_t n, const double *p, const double *bv,
                           const double *dot, double *x, hipStream_t st);
// x = B^T q + cv * dot[0] (q of length m, x of length n).
hipError_t launch_bhu_btmul(const double *d, const double *e, int64_t n, const double *q, const double *cv,
                            const double *dot, double *x, hipStream_t st);

// Reflector for a[off .. len): writes the leading value to *alpha and the
// unit essential vector (zero outside [off, len)) to y[0 .. len); the
// identity (y = 0, *alpha = a[off]) when a[off+1 .. len) is all zero.
hipError_t launch_bhu_house(const double *a, int64_t off, int64_t len, double *alpha, double *y, hipStream_t st);

// dst[i] = src[i] (src null: 0) for i < count.
hipError_t launch_bhu_copy(double *dst, const double *src, int64_t count, hipStream_t st);

// C = beta C + alpha A op(B): A m x K (lda), op(B) = B (K x n, ldb) or, with
// transb, B^T (B stored n x K, ldb); C m x n (ldc).  FP64 matrix cores, one
// wavefront per 64 x 64 block of C.
hipError_t launch_bhu_gemm(const double *A, int64_t lda, const double *B, int64_t ldb, bool transb, double *C,
                           int64_t ldc, int64_t m, int64_t n, int64_t K, double alpha, double beta, hipStream_t st);

}  // namespace bdu
