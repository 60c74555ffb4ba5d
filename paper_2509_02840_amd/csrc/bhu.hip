// bhu.hip -- gfx950 kernels of the Householder bidiagonal update (Section
// 3.3, Theorem 1, Algorithm 1).  Each step of the algorithm needs column k
// (then row k) of Q_i^T (B + b c^T) P_j, never formed: it is reached through
// matrix-vector products with the reflector collections Y (m x i), W (n x j)
// and the explicit inverses S = T^{-1}, Rv = R^{-1} of the unit upper
// triangular matrices of eq. (TR).  Those products stream Y, W, S and Rv and
// are bound by memory bandwidth; the products with Q and P at the end are
// dense contractions and run on the FP64 matrix cores.
#include <hip/hip_runtime.h>

#include "bhu.h"

namespace bdu {

namespace {

typedef double acc4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void bhu_gemv_t_kernel(const double *X, int64_t ld, int64_t rows, const double *v,
                                                         double alpha, double *out)
{
    const int64_t c = blockIdx.x;
    const double *col = X + c * ld;
    double s = 0.0;
    for (int64_t r = threadIdx.x; r < rows; r += 256) s = fma(col[r], v[r], s);
    __shared__ double red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = alpha * red[0];
}

// Two passes, so that a few thousand rows still spread over the chip.
// Pass 1: block (rb, ch) sums columns [ch K, ch K + K) of rows [64 rb, 64 rb + 64)
// (wavefront g takes columns g, g + 4, ...; lane = row, so every column read
// is 512 contiguous bytes) into part[ch lp + r].  Pass 2 adds the chunks in
// order.
constexpr int kChunk = 128;

__global__ __launch_bounds__(256) void bhu_gemv_n_part_kernel(const double *X, int64_t ld, int64_t rows,
                                                               int64_t cols, const double *h, int64_t hs,
                                                               double *part, int64_t lp)
{
    const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int64_t r = (int64_t)blockIdx.x * 64 + lane;
    const int64_t c0 = (int64_t)blockIdx.y * kChunk;
    const int64_t c1 = c0 + kChunk < cols ? c0 + kChunk : cols;
    double s = 0.0;
    if (r < rows)
        for (int64_t c = c0 + g; c < c1; c += 4) s = fma(X[r + c * ld], h[c * hs], s);
    __shared__ double red[4][64];
    red[g][lane] = s;
    __syncthreads();
    if (g == 0 && r < rows) part[blockIdx.y * lp + r] = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
}

__global__ __launch_bounds__(256) void bhu_gemv_n_sum_kernel(const double *part, int64_t lp, int64_t nch,
                                                             int64_t rows, double alpha, const double *base,
                                                             int64_t unit, double *out)
{
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= rows) return;
    double t = 0.0;
    for (int64_t q = 0; q < nch; ++q) t += part[q * lp + r];
    const double b0 = (base ? base[r] : 0.0) + (r == unit ? 1.0 : 0.0);
    out[r] = fma(alpha, t, b0);
}

__global__ __launch_bounds__(256) void bhu_bmul_kernel(const double *d, const double *e, int64_t m, int64_t n,
                                                       const double *p, const double *bv, const double *dot,
                                                       double *x)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= m) return;
    double s = 0.0;
    if (i < n) s = d[i] * p[i];
    if (i + 1 < n) s = fma(e[i], p[i + 1], s);
    x[i] = fma(bv[i], dot[0], s);
}

__global__ __launch_bounds__(256) void bhu_btmul_kernel(const double *d, const double *e, int64_t n, const double *q,
                                                        const double *cv, const double *dot, double *x)
{
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    double s = d[j] * q[j];
    if (j > 0) s = fma(e[j - 1], q[j - 1], s);
    x[j] = fma(cv[j], dot[0], s);
}

__global__ __launch_bounds__(1024) void bhu_house_kernel(const double *a, int64_t off, int64_t len, double *alpha,
                                                         double *y)
{
    __shared__ double ss[1024];
    __shared__ int nz[1024];
    __shared__ double scal[2];  // y[off] and the divisor (0: identity)
    double s = 0.0;
    int f = 0;
    for (int64_t t = off + 1 + threadIdx.x; t < len; t += 1024) {
        const double v = a[t];
        s = fma(v, v, s);
        f |= v != 0.0;
    }
    ss[threadIdx.x] = s;
    nz[threadIdx.x] = f;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            ss[threadIdx.x] += ss[threadIdx.x + w];
            nz[threadIdx.x] |= nz[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double x0 = a[off], sigma = ss[0];
        if (!nz[0]) {
            *alpha = x0;
            scal[0] = 0.0;
            scal[1] = 0.0;
        } else {
            const double nrm = sqrt(fma(x0, x0, sigma));
            const double al = x0 >= 0.0 ? -nrm : nrm;
            const double y0 = x0 - al;
            const double yn = sqrt(fma(y0, y0, sigma));
            *alpha = al;
            scal[0] = y0 / yn;
            scal[1] = yn;
        }
    }
    __syncthreads();
    const double y0 = scal[0], yn = scal[1];
    for (int64_t t = threadIdx.x; t < len; t += 1024) {
        double v = 0.0;
        if (yn != 0.0) v = t == off ? y0 : (t > off ? a[t] / yn : 0.0);
        y[t] = v;
    }
}

__global__ __launch_bounds__(256) void bhu_copy_kernel(double *dst, const double *src, int64_t count)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < count) dst[i] = src ? src[i] : 0.0;
}

// v_mfma_f64_16x16x4f64: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]
// and holds D[l / 16 + 4 q][l % 16] in element q of its accumulator.
template <bool TB>
__global__ __launch_bounds__(64) void bhu_gemm_kernel(const double *A, int64_t lda, const double *B, int64_t ldb,
                                                      double *C, int64_t ldc, int64_t m, int64_t n, int64_t K,
                                                      double alpha, double beta)
{
    const int l = threadIdx.x, rr = l / 16, cc = l % 16;
    const int64_t R0 = (int64_t)blockIdx.x * 64, J0 = (int64_t)blockIdx.y * 64;
    acc4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = acc4{0.0, 0.0, 0.0, 0.0};
    for (int64_t c0 = 0; c0 < K; c0 += 4) {
        const int64_t c = c0 + rr;
        double av[4], bv[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int64_t i = R0 + 16 * t + cc, j = J0 + 16 * t + cc;
            av[t] = (c < K && i < m) ? A[i + c * lda] : 0.0;
            bv[t] = (c < K && j < n) ? (TB ? B[j + c * ldb] : B[c + j * ldb]) : 0.0;
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t i = R0 + 16 * a + rr + 4 * q, j = J0 + 16 * b + cc;
                if (i >= m || j >= n) continue;
                const double v = alpha * acc[a][b][q];
                C[i + j * ldc] = beta == 0.0 ? v : fma(beta, C[i + j * ldc], v);
            }
}

}  // namespace

hipError_t launch_bhu_gemv_t(const double *X, int64_t ld, int64_t rows, int64_t cols, const double *v, double alpha,
                             double *out, hipStream_t st)
{
    if (cols <= 0) return hipSuccess;
    hipLaunchKernelGGL(bhu_gemv_t_kernel, dim3((unsigned)cols), dim3(256), 0, st, X, ld, rows, v, alpha, out);
    return hipGetLastError();
}

hipError_t launch_bhu_gemv_n(const double *X, int64_t ld, int64_t rows, int64_t cols, const double *h, int64_t hs,
                             double alpha, const double *base, int64_t unit, double *out, double *part, int64_t lp,
                             hipStream_t st)
{
    if (rows <= 0) return hipSuccess;
    if (rows > lp) return hipErrorInvalidValue;
    const int64_t nch = (cols + kChunk - 1) / kChunk;
    if (nch > 0)
        hipLaunchKernelGGL(bhu_gemv_n_part_kernel, dim3((unsigned)((rows + 63) / 64), (unsigned)nch), dim3(256), 0,
                           st, X, ld, rows, cols, h, hs, part, lp);
    hipLaunchKernelGGL(bhu_gemv_n_sum_kernel, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, st,
                       (const double *)part, lp, nch, rows, alpha, base, unit, out);
    return hipGetLastError();
}

hipError_t launch_bhu_bmul(const double *d, const double *e, int64_t m, int64_t n, const double *p, const double *bv,
                           const double *dot, double *x, hipStream_t st)
{
    hipLaunchKernelGGL(bhu_bmul_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, d, e, m, n, p, bv, dot,
                       x);
    return hipGetLastError();
}

hipError_t launch_bhu_btmul(const double *d, const double *e, int64_t n, const double *q, const double *cv,
                            const double *dot, double *x, hipStream_t st)
{
    hipLaunchKernelGGL(bhu_btmul_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, d, e, n, q, cv, dot, x);
    return hipGetLastError();
}

hipError_t launch_bhu_house(const double *a, int64_t off, int64_t len, double *alpha, double *y, hipStream_t st)
{
    if (off < 0 || off >= len) return hipErrorInvalidValue;
    hipLaunchKernelGGL(bhu_house_kernel, dim3(1), dim3(1024), 0, st, a, off, len, alpha, y);
    return hipGetLastError();
}

hipError_t launch_bhu_copy(double *dst, const double *src, int64_t count, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(bhu_copy_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, dst, src, count);
    return hipGetLastError();
}

hipError_t launch_bhu_gemm(const double *A, int64_t lda, const double *B, int64_t ldb, bool transb, double *C,
                           int64_t ldc, int64_t m, int64_t n, int64_t K, double alpha, double beta, hipStream_t st)
{
    if (m <= 0 || n <= 0) return hipSuccess;
    const dim3 grid((unsigned)((m + 63) / 64), (unsigned)((n + 63) / 64));
    if (transb)
        hipLaunchKernelGGL(bhu_gemm_kernel<true>, grid, dim3(64), 0, st, A, lda, B, ldb, C, ldc, m, n, K, alpha, beta);
    else
        hipLaunchKernelGGL(bhu_gemm_kernel<false>, grid, dim3(64), 0, st, A, lda, B, ldb, C, ldc, m, n, K, alpha,
                           beta);
    return hipGetLastError();
}

}  // namespace bdu
