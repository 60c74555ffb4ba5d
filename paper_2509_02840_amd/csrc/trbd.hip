// trbd.hip -- gfx950 kernels of the truncated bidiagonal approximation
// (Section 1.3, eqs. (trBD), (errtrBD)): A = Q Bd P^T is approximated by the r
// columns i of Bd with the largest t_i = d_i^2 + e_{i-1}^2 (e_0 = 0), as
// A_r = Qr Pr^T with Qr(:, j) = d_i q_i + e_{i-1} q_{i-1}, Pr(:, j) = p_i;
// the squared error is the sum of the dropped t_i.  Every product and sum is
// rounded on its own (-ffp-contract=off).
#include <hip/hip_runtime.h>

#include "trbd.h"

namespace bdu {

__global__ __launch_bounds__(256) void trbd_t_kernel(const double *d, const double *e, int64_t n, double *t)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double sq = d[i] * d[i];
    t[i] = i == 0 ? sq : sq + e[i - 1] * e[i - 1];
}

// rank_i = #{j : t_j > t_i, or t_j == t_i and j < i}: the position of i in a
// stable sort by decreasing t; the first r positions are the kept columns.
__global__ __launch_bounds__(256) void trbd_rank_kernel(const double *t, int64_t n, int64_t r, int64_t *rank,
                                                        int64_t *idx)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double ti = t[i];
    int64_t k = 0;
    for (int64_t j = 0; j < n; ++j) {
        const double tj = t[j];
        k += (tj > ti || (tj == ti && j < i)) ? 1 : 0;
    }
    rank[i] = k;
    if (k < r) idx[k] = i;
}

// err2 = sum of the dropped t_i, i ascending, from 0 (one lane).
__global__ void trbd_err_kernel(const double *t, const int64_t *rank, int64_t n, int64_t r, double *err2)
{
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i)
        if (rank[i] >= r) s = s + t[i];
    err2[0] = s;
}

// grid (ceil(max(m, n) / 256), r): Qr(:, j) and Pr(:, j), one lane per row.
__global__ __launch_bounds__(256) void trbd_form_kernel(const double *Q, int64_t ldq, int64_t m, const double *P,
                                                        int64_t ldp, int64_t n, const double *d, const double *e,
                                                        const int64_t *idx, double *Qr, double *Pr)
{
    const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t j = blockIdx.y;
    const int64_t i = idx[j];
    if (row < m) {
        const double a = d[i] * Q[row + i * ldq];
        Qr[row + j * m] = i == 0 ? a : a + e[i - 1] * Q[row + (i - 1) * ldq];
    }
    if (row < n) Pr[row + j * n] = P[row + i * ldp];
}

hipError_t launch_trbd(const double *Q, int64_t ldq, int64_t m, const double *P, int64_t ldp, int64_t n,
                       const double *d, const double *e, int64_t r, double *t, int64_t *rank, int64_t *idx,
                       double *err2, double *Qr, double *Pr, hipStream_t st)
{
    if (r < 1 || r > n || r > 65535) return hipErrorInvalidValue;
    const unsigned gn = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(trbd_t_kernel, dim3(gn), dim3(256), 0, st, d, e, n, t);
    hipLaunchKernelGGL(trbd_rank_kernel, dim3(gn), dim3(256), 0, st, (const double *)t, n, r, rank, idx);
    hipLaunchKernelGGL(trbd_err_kernel, dim3(1), dim3(64), 0, st, (const double *)t, (const int64_t *)rank, n, r,
                       err2);
    const int64_t rows = m > n ? m : n;
    hipLaunchKernelGGL(trbd_form_kernel, dim3((unsigned)((rows + 255) / 256), (unsigned)r), dim3(256), 0, st, Q, ldq,
                       m, P, ldp, n, d, e, (const int64_t *)idx, Qr, Pr);
    return hipGetLastError();
}

}  // namespace bdu
