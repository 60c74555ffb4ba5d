// orth.hip -- gfx950 kernels of the orthogonality monitor and correction
// (the paper reorthogonalizes its factors a few times over a stream; this is
// the dense-contraction part of the method, so it runs on the FP64 matrix
// cores: v_mfma_f64_16x16x4f64, one wavefront per 64 x 64 output block).
//
// Operand layout of v_mfma_f64_16x16x4f64 (D = A B + C, A 16 x 4, B 4 x 16):
// lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16] and holds
// D[l / 16 + 4 q][l % 16] in element q of its 4-double accumulator.
#include <hip/hip_runtime.h>

#include "orth.h"

namespace bdu {

typedef double mfma_acc __attribute__((ext_vector_type(4)));

// E = X^T X - I on the blocks at or above the diagonal, each entry also
// written to its mirror, so E is exactly symmetric.  grid (nb, nb), nb =
// lde / 64; the contraction runs over the ld rows (padding rows are zero).
// The MFMA operands run across columns of X, so 16-row x 64-column tiles of
// X are loaded down the columns (16 consecutive doubles per 16 lanes) into
// LDS, the next tile's loads in flight while the current one is multiplied.
// A tile column is 34 doubles apart: a 32-lane half of an operand read
// (columns c = 0..15, rows r and r+1) then meets 32 distinct bank pairs.
constexpr int kGramRows = 16, kGramPad = 34;

__global__ __launch_bounds__(64) void orth_gram_kernel(const double *X, int64_t ld, int64_t k, double *E,
                                                       int64_t lde)
{
    __shared__ double ta[64 * kGramPad], tb[64 * kGramPad];
    const int bi = blockIdx.x, bj = blockIdx.y;
    if (bj < bi) return;
    const int l = threadIdx.x, rr = l / 16, cc = l % 16;
    const int64_t I0 = (int64_t)bi * 64, J0 = (int64_t)bj * 64;
    mfma_acc acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = mfma_acc{0.0, 0.0, 0.0, 0.0};
    // load q of a tile: row cc, column 4 q + rr of the 64-column block
    double pa[16], pb[16];
    auto load = [&](int64_t r0) {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int64_t ci = I0 + 4 * q + rr, cj = J0 + 4 * q + rr;
            pa[q] = ci < k ? X[(r0 + cc) + ci * ld] : 0.0;
            pb[q] = cj < k ? X[(r0 + cc) + cj * ld] : 0.0;
        }
    };
    load(0);
    for (int64_t r0 = 0; r0 < ld; r0 += kGramRows) {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            ta[(4 * q + rr) * kGramPad + cc] = pa[q];
            tb[(4 * q + rr) * kGramPad + cc] = pb[q];
        }
        if (r0 + kGramRows < ld) load(r0 + kGramRows);
        __syncthreads();
#pragma unroll
        for (int s4 = 0; s4 < kGramRows / 4; ++s4) {
            double av[4], bv[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                av[t] = ta[(16 * t + cc) * kGramPad + 4 * s4 + rr];
                bv[t] = tb[(16 * t + cc) * kGramPad + 4 * s4 + rr];
            }
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t i = I0 + 16 * a + rr + 4 * q, j = J0 + 16 * b + cc;
                if (i >= k || j >= k || (bi == bj && i > j)) continue;
                const double v = acc[a][b][q] - (i == j ? 1.0 : 0.0);
                E[i + j * lde] = v;
                E[j + i * lde] = v;
            }
}

// part[j] = sum_i E(i, j)^2 over the k rows of column j (one block of 256
// lanes per column, a fixed tree), then out[0] = sqrt(sum_j part[j]).
__global__ __launch_bounds__(256) void orth_colsq_kernel(const double *E, int64_t k, int64_t lde, double *part)
{
    __shared__ double red[256];
    const int64_t j = blockIdx.x;
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < k; i += 256) s = fma(E[i + j * lde], E[i + j * lde], s);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[j] = red[0];
}

__global__ __launch_bounds__(256) void orth_sum_kernel(const double *part, int64_t k, double *out)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t j = threadIdx.x; j < k; j += 256) s += part[j];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sqrt(red[0]);
}

// Y = X - (X E) / 2.  E is symmetric, so the B operand E(c, j) is read as
// E(j, c): both operands then run down columns.  grid (ld / 64, lde / 64).
__global__ __launch_bounds__(64) void orth_update_kernel(const double *X, int64_t ld, int64_t k, const double *E,
                                                         int64_t lde, double *Y)
{
    const int l = threadIdx.x, rr = l / 16, cc = l % 16;
    const int64_t R0 = (int64_t)blockIdx.x * 64, J0 = (int64_t)blockIdx.y * 64;
    mfma_acc acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = mfma_acc{0.0, 0.0, 0.0, 0.0};
    for (int64_t c0 = 0; c0 < k; c0 += 4) {
        const int64_t c = c0 + rr;
        double av[4], bv[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int64_t j = J0 + 16 * t + cc;
            av[t] = c < k ? X[(R0 + 16 * t + cc) + c * ld] : 0.0;
            bv[t] = (c < k && j < k) ? E[j + c * lde] : 0.0;
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
                if (j >= k) continue;
                Y[i + j * ld] = X[i + j * ld] - 0.5 * acc[a][b][q];
            }
}

hipError_t launch_orth_gram(const double *X, int64_t ld, int64_t k, double *E, int64_t lde, hipStream_t st)
{
    if (ld % 128 || lde % 64 || lde < k || k < 1) return hipErrorInvalidValue;  // ld: whole 16-row tiles
    const unsigned nb = (unsigned)(lde / 64);
    hipLaunchKernelGGL(orth_gram_kernel, dim3(nb, nb), dim3(64), 0, st, X, ld, k, E, lde);
    return hipGetLastError();
}

hipError_t launch_orth_norm(const double *E, int64_t k, int64_t lde, double *part, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(orth_colsq_kernel, dim3((unsigned)k), dim3(256), 0, st, E, k, lde, part);
    hipLaunchKernelGGL(orth_sum_kernel, dim3(1), dim3(256), 0, st, (const double *)part, k, out);
    return hipGetLastError();
}

hipError_t launch_orth_update(const double *X, int64_t ld, int64_t k, const double *E, int64_t lde, double *Y,
                              hipStream_t st)
{
    if (ld % 128 || lde % 64 || lde < k || k < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(orth_update_kernel, dim3((unsigned)(ld / 64), (unsigned)(lde / 64)), dim3(64), 0, st, X, ld,
                       k, E, lde, Y);
    return hipGetLastError();
}

}  // namespace bdu
