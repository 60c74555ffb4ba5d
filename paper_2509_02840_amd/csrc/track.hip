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

// Row sums over a tracked basis run in chunks of kTrackChunk rows: a
// sequential fma from 0 inside a chunk (rows ascending), then the chunk
// partials added in ascending order from 0.

// part[side][k][j] = sum over the rows i of chunk k of A(i, j) x_i.  grid
// (chunks, ceil(cols / 64), 2 sides), one lane per column j; each lane runs
// down its own column, 32 loads ahead.
__global__ __launch_bounds__(64) void track_partial_kernel(TrackSides s, double *part, int64_t nchunk)
{
    const TrackSide &t = s.side[blockIdx.z];
    const int64_t i0 = (int64_t)blockIdx.x * kTrackChunk;
    const int64_t j = (int64_t)blockIdx.y * 64 + threadIdx.x;
    if (i0 >= t.rows || j >= t.cols) return;
    const int64_t i1 = i0 + kTrackChunk < t.rows ? i0 + kTrackChunk : t.rows;
    const double *a = t.A + j * t.lda;
    double p = 0.0;
    int64_t i = i0;
    for (; i + 32 <= i1; i += 32) {
        double av[32], xv[32];
#pragma unroll
        for (int q = 0; q < 32; ++q) {
            av[q] = a[i + q];
            xv[q] = t.x[i + q];
        }
#pragma unroll
        for (int q = 0; q < 32; ++q) p = fma(av[q], xv[q], p);
    }
    for (; i < i1; ++i) p = fma(a[i], t.x[i], p);
    part[((int64_t)blockIdx.z * nchunk + blockIdx.x) * t.cols + j] = p;
}

// xhat_j = sum over chunks k (ascending) of part[side][k][j], from 0.
// grid (ceil(cols / 64), 2 sides).
__global__ __launch_bounds__(64) void track_combine_kernel(TrackSides s, const double *part, int64_t nchunk)
{
    const TrackSide &t = s.side[blockIdx.y];
    const int64_t j = (int64_t)blockIdx.x * 64 + threadIdx.x;
    if (j >= t.cols) return;
    const int64_t nk = (t.rows + kTrackChunk - 1) / kTrackChunk;
    double total = 0.0;
    for (int64_t k = 0; k < nk; ++k) total = total + part[((int64_t)blockIdx.y * nchunk + k) * t.cols + j];
    t.xhat[j] = total;
}

// xperp_i = x_i - s_i, s_i = sum_j A(i, j) xhat_j (fma, j ascending); one
// block per chunk of rows, one lane per row; lane 0 then sums the chunk's
// xperp_i^2 in row order (fma from 0) into npart[side][chunk].
// grid (chunks, 2 sides), kTrackChunk lanes.
__global__ __launch_bounds__(kTrackChunk) void track_residual_kernel(TrackSides s, double *npart, int64_t nchunk)
{
    __shared__ double sq[kTrackChunk];
    const TrackSide &t = s.side[blockIdx.y];
    const int64_t i0 = (int64_t)blockIdx.x * kTrackChunk;
    if (i0 >= t.rows) return;
    const int64_t i = i0 + threadIdx.x;
    double xp = 0.0;
    if (i < t.rows) {
        double acc = 0.0;
        for (int64_t j = 0; j < t.cols; ++j) acc = fma(t.A[i + j * t.lda], t.xhat[j], acc);
        xp = t.x[i] - acc;
        t.xperp[i] = xp;
    }
    sq[threadIdx.x] = xp;
    __syncthreads();
    if (threadIdx.x == 0) {
        const int cnt = t.rows - i0 < kTrackChunk ? (int)(t.rows - i0) : kTrackChunk;
        double p = 0.0;
        for (int q = 0; q < cnt; ++q) p = fma(sq[q], sq[q], p);
        npart[(int64_t)blockIdx.y * nchunk + blockIdx.x] = p;
    }
}

// norm = sqrt(sum over chunks (ascending, from 0) of npart): lane 0 for
// side 0, lane 1 for side 1.  The norm becomes the last entry of the middle
// update vector and is copied to norms[side].
__global__ __launch_bounds__(64) void track_norm_kernel(TrackSides s, const double *npart, int64_t nchunk,
                                                        double *norms)
{
    const int side = threadIdx.x;
    if (side > 1) return;
    const TrackSide &t = s.side[side];
    const int64_t nk = (t.rows + kTrackChunk - 1) / kTrackChunk;
    double total = 0.0;
    for (int64_t k = 0; k < nk; ++k) total = total + npart[(int64_t)side * nchunk + k];
    const double nrm = sqrt(total);
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

hipError_t launch_track_project(const TrackSides &s, int64_t max_rows, int64_t r, double *part, hipStream_t st)
{
    const int64_t nchunk = (max_rows + kTrackChunk - 1) / kTrackChunk;
    hipLaunchKernelGGL(track_partial_kernel, dim3((unsigned)nchunk, (unsigned)((r + 63) / 64), 2), dim3(64), 0, st, s,
                       part, nchunk);
    hipLaunchKernelGGL(track_combine_kernel, dim3((unsigned)((r + 63) / 64), 2), dim3(64), 0, st, s,
                       (const double *)part, nchunk);
    return hipGetLastError();
}

hipError_t launch_track_complement(const TrackSides &s, int64_t max_rows, double *npart, double *norms,
                                   hipStream_t st)
{
    const int64_t nchunk = (max_rows + kTrackChunk - 1) / kTrackChunk;
    hipLaunchKernelGGL(track_residual_kernel, dim3((unsigned)nchunk, 2), dim3(kTrackChunk), 0, st, s, npart, nchunk);
    hipLaunchKernelGGL(track_norm_kernel, dim3(1), dim3(64), 0, st, s, (const double *)npart, nchunk, norms);
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
