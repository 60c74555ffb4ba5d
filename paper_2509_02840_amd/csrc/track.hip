// track.hip -- gfx950 kernels of the subspace-tracking update (Brust &
// Saunders, Section 4, eqs. (lrup)-(bdlrup)): projections of b and c onto the
// tracked bases and their complements, the middle matrix's inputs, the
// truncation of the updated bidiagonal and the thin products.  The middle
// (r+1) x (r+1) update itself is an ordinary BGU handle.  FP64; every sum is
// a sequential fma in a stated order.
#include <hip/hip_runtime.h>

#include "primitives.h"
#include "track.h"

namespace bdu {

// y_j = sum_i A(i, j) x_i, acc = fma(A(i, j), x_i, acc), i ascending from 0.
// One lane per output column; 64 x 64 tiles of A pass through LDS so that
// the global reads run down the columns.  grid (ceil(cols / 64), 2 sides).
__global__ __launch_bounds__(64) void track_project_kernel(TrackSides s)
{
    __shared__ double tile[64][65];
    __shared__ double xs[64];
    const TrackSide &t = s.side[blockIdx.y];
    const int lane = threadIdx.x;
    const int64_t j0 = (int64_t)blockIdx.x * 64;
    if (j0 >= t.cols) return;
    const int64_t j = j0 + lane;
    double acc = 0.0;
    for (int64_t i0 = 0; i0 < t.rows; i0 += 64) {
        const int64_t i = i0 + lane;
        for (int c = 0; c < 64; ++c)
            tile[c][lane] = (i < t.rows && j0 + c < t.cols) ? t.A[i + (j0 + c) * t.lda] : 0.0;
        xs[lane] = i < t.rows ? t.x[i] : 0.0;
        __syncthreads();
        const int nr = t.rows - i0 < 64 ? (int)(t.rows - i0) : 64;
        for (int k = 0; k < nr; ++k) acc = fma(tile[lane][k], xs[k], acc);
        __syncthreads();
    }
    if (j < t.cols) t.xhat[j] = acc;
}

// xperp_i = x_i - s_i, s_i = sum_j A(i, j) xhat_j (fma, j ascending).
// grid (ceil(rows / 256), 2 sides), 256 lanes, one per row.
__global__ __launch_bounds__(256) void track_residual_kernel(TrackSides s)
{
    const TrackSide &t = s.side[blockIdx.y];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= t.rows) return;
    double acc = 0.0;
    for (int64_t j = 0; j < t.cols; ++j) acc = fma(t.A[i + j * t.lda], t.xhat[j], acc);
    t.xperp[i] = t.x[i] - acc;
}

// norm = sqrt(sum_i xperp_i^2), acc = fma(xperp_i, xperp_i, acc), i
// ascending: lane 0 for side 0, lane 1 for side 1.  The norm becomes the
// last entry of the middle update vector and is copied to norms[side].
__global__ __launch_bounds__(64) void track_norm_kernel(TrackSides s, double *norms)
{
    const int side = threadIdx.x;
    if (side > 1) return;
    const TrackSide &t = s.side[side];
    double acc = 0.0;
    for (int64_t i = 0; i < t.rows; ++i) acc = fma(t.xperp[i], t.xperp[i], acc);
    const double nrm = sqrt(acc);
    t.xhat[t.cols] = nrm;
    norms[side] = nrm;
}

// w_i = xperp_i / norm (in place).  grid (ceil(rows / 256), 2 sides).
__global__ __launch_bounds__(256) void track_scale_kernel(TrackSides s)
{
    const TrackSide &t = s.side[blockIdx.y];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= t.rows) return;
    t.xperp[i] = t.xperp[i] / t.xhat[t.cols];
}

// The middle factorization before its update: Q = P = I (R x R, leading
// dimensions ldq, ldp), d = [d; 0], e = [e; 0].  grid (R), R <= 1024 lanes.
__global__ void track_reset_kernel(TrackMiddle mid, const double *d, const double *e)
{
    const int col = blockIdx.x;
    for (int i = threadIdx.x; i < mid.R; i += blockDim.x) {
        mid.Q[i + (int64_t)col * mid.ldq] = i == col ? 1.0 : 0.0;
        mid.P[i + (int64_t)col * mid.ldp] = i == col ? 1.0 : 0.0;
    }
    if (col == 0)
        for (int i = threadIdx.x; i < mid.R; i += blockDim.x) {
            mid.d[i] = i < mid.R - 1 ? d[i] : 0.0;
            if (i < mid.R - 1) mid.e[i] = i < mid.R - 2 ? e[i] : 0.0;
        }
}

// Drop the row and column k of the updated R x R bidiagonal with the
// smallest column norm (d_k^2 + e_{k-1}^2 as fma(d_k, d_k, e_{k-1} e_{k-1});
// ties drop the highest k): d, e of the tracked factorization become the
// kept entries, with 0 joining k-1 and k+1.  One lane.
__global__ void track_truncate_kernel(TrackMiddle mid, double *d, double *e, int *kdrop)
{
    if (threadIdx.x != 0) return;
    const int R = mid.R;
    int k = R - 1;
    double best = fma(mid.d[R - 1], mid.d[R - 1], mid.e[R - 2] * mid.e[R - 2]);
    for (int j = R - 2; j >= 0; --j) {
        const double nj = j == 0 ? mid.d[0] * mid.d[0] : fma(mid.d[j], mid.d[j], mid.e[j - 1] * mid.e[j - 1]);
        if (nj < best) {
            best = nj;
            k = j;
        }
    }
    *kdrop = k;
    for (int j = 0; j < R - 1; ++j) d[j] = mid.d[j < k ? j : j + 1];
    for (int j = 0; j + 1 < R - 1; ++j) {
        const int a = j < k ? j : j + 1, b = j + 1 < k ? j + 1 : j + 2;
        e[j] = b == a + 1 ? mid.e[a] : 0.0;
    }
}

// out(i, j) = sum_{l < r} A(i, l) M(l, kj) + w_i M(r, kj), each term an fma
// in that order, kj = j for j < k and j + 1 otherwise (M = the middle Q for
// side 0, P for side 1).  grid (ceil(rows / 256), r, 2 sides).
__global__ __launch_bounds__(256) void track_product_kernel(TrackSides s, TrackMiddle mid, const int *kdrop,
                                                            double *out0, double *out1)
{
    const TrackSide &t = s.side[blockIdx.z];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= t.rows) return;
    const int j = blockIdx.y;
    const int k = *kdrop;
    const int kj = j < k ? j : j + 1;
    const double *M = blockIdx.z == 0 ? mid.Q + (int64_t)kj * mid.ldq : mid.P + (int64_t)kj * mid.ldp;
    double acc = 0.0;
    for (int64_t l = 0; l < t.cols; ++l) acc = fma(t.A[i + l * t.lda], M[l], acc);
    acc = fma(t.xperp[i], M[t.cols], acc);
    (blockIdx.z == 0 ? out0 : out1)[i + (int64_t)j * t.lda] = acc;
}

hipError_t launch_track_project(const TrackSides &s, int64_t max_rows, int64_t r, hipStream_t st)
{
    (void)max_rows;
    hipLaunchKernelGGL(track_project_kernel, dim3((unsigned)((r + 63) / 64), 2), dim3(64), 0, st, s);
    return hipGetLastError();
}

hipError_t launch_track_complement(const TrackSides &s, int64_t max_rows, double *norms, hipStream_t st)
{
    const dim3 g((unsigned)((max_rows + 255) / 256), 2);
    hipLaunchKernelGGL(track_residual_kernel, g, dim3(256), 0, st, s);
    hipLaunchKernelGGL(track_norm_kernel, dim3(1), dim3(64), 0, st, s, norms);
    return hipGetLastError();
}

hipError_t launch_track_scale(const TrackSides &s, int64_t max_rows, hipStream_t st)
{
    hipLaunchKernelGGL(track_scale_kernel, dim3((unsigned)((max_rows + 255) / 256), 2), dim3(256), 0, st, s);
    return hipGetLastError();
}

hipError_t launch_track_reset(const TrackMiddle &mid, const double *d, const double *e, hipStream_t st)
{
    hipLaunchKernelGGL(track_reset_kernel, dim3(mid.R), dim3(mid.R < 1024 ? ((mid.R + 63) / 64) * 64 : 1024), 0, st,
                       mid, d, e);
    return hipGetLastError();
}

hipError_t launch_track_finish(const TrackSides &s, const TrackMiddle &mid, double *d, double *e, int *kdrop,
                               int64_t max_rows, int64_t r, double *out0, double *out1, hipStream_t st)
{
    hipLaunchKernelGGL(track_truncate_kernel, dim3(1), dim3(64), 0, st, mid, d, e, kdrop);
    hipLaunchKernelGGL(track_product_kernel, dim3((unsigned)((max_rows + 255) / 256), (unsigned)r, 2), dim3(256), 0,
                       st, s, mid, kdrop, out0, out1);
    return hipGetLastError();
}

}  // namespace bdu
