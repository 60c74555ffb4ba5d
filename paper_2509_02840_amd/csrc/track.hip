// track.hip -- gfx950 kernels of the subspace-tracking update (Brust &
// Saunders, Section 4, eqs. (lrup)-(bdlrup) and the unaugmented case after
// them): projections of b and c onto the tracked bases and their
// complements, the middle matrix's inputs, the truncation of the updated
// bidiagonal and the thin products.  The middle update itself is an
// ordinary BGU handle.  FP64; every sum is a sequential fma in a stated
// order.
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
// block per chunk of rows, one lane per row (x may be xperp itself: each
// lane reads its entry before writing it); lane 0 then sums the chunk's
// x_i^2 and xperp_i^2 in row order (fma from 0) into npart[side][chunk].
// grid (chunks, 2 sides), kTrackChunk lanes.
__global__ __launch_bounds__(kTrackChunk) void track_residual_kernel(TrackSides s, double *npart, int64_t nchunk)
{
    __shared__ double sq[kTrackChunk], sx[kTrackChunk];
    const TrackSide &t = s.side[blockIdx.y];
    const int64_t i0 = (int64_t)blockIdx.x * kTrackChunk;
    if (i0 >= t.rows) return;
    const int64_t i = i0 + threadIdx.x;
    double xp = 0.0, xv = 0.0;
    if (i < t.rows) {
        double acc = 0.0;
        for (int64_t j = 0; j < t.cols; ++j) acc = fma(t.A[i + j * t.lda], t.xhat[j], acc);
        xv = t.x[i];
        xp = xv - acc;
        t.xperp[i] = xp;
    }
    sq[threadIdx.x] = xp;
    sx[threadIdx.x] = xv;
    __syncthreads();
    if (threadIdx.x == 0) {
        const int cnt = t.rows - i0 < kTrackChunk ? (int)(t.rows - i0) : kTrackChunk;
        double p = 0.0, px = 0.0;
        for (int q = 0; q < cnt; ++q) {
            px = fma(sx[q], sx[q], px);
            p = fma(sq[q], sq[q], p);
        }
        npart[2 * ((int64_t)blockIdx.y * nchunk + blockIdx.x)] = px;
        npart[2 * ((int64_t)blockIdx.y * nchunk + blockIdx.x) + 1] = p;
    }
}

// sums[2 side] = x^T x, sums[2 side + 1] = xperp^T xperp: the chunk
// partials added in ascending order from 0.  Lanes 0 and 1: the two sides.
__global__ __launch_bounds__(64) void track_sums_kernel(TrackSides s, const double *npart, int64_t nchunk,
                                                        double *sums)
{
    const int side = threadIdx.x;
    if (side > 1) return;
    const TrackSide &t = s.side[side];
    const int64_t nk = (t.rows + kTrackChunk - 1) / kTrackChunk;
    double tx = 0.0, tp = 0.0;
    for (int64_t k = 0; k < nk; ++k) {
        tx = tx + npart[2 * ((int64_t)side * nchunk + k)];
        tp = tp + npart[2 * ((int64_t)side * nchunk + k) + 1];
    }
    sums[2 * side] = tx;
    sums[2 * side + 1] = tp;
}

// xhat += add for the sides in mask (bit side).  grid (ceil(cols / 64), 2).
__global__ __launch_bounds__(64) void track_accumulate_kernel(TrackSides s, const double *add, int64_t r, int mask)
{
    const int side = blockIdx.y;
    if (!((mask >> side) & 1)) return;
    const int64_t j = (int64_t)blockIdx.x * 64 + threadIdx.x;
    if (j >= r) return;
    s.side[side].xhat[j] = s.side[side].xhat[j] + add[side * r + j];
}

// w_i = xperp_i / norm (in place) for each side with a positive norm.
// grid (ceil(rows / 256), 2 sides).
__global__ __launch_bounds__(256) void track_scale_kernel(TrackSides s, double delta, double gamma)
{
    const TrackSide &t = s.side[blockIdx.y];
    const double nrm = blockIdx.y == 0 ? delta : gamma;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (!(nrm > 0.0) || i >= t.rows) return;
    t.xperp[i] = t.xperp[i] / nrm;
}

// The middle factorization before its pass: Q = I (pm x pm, leading
// dimension ldq), P = I (pn x pn), and
//   not flipped: d = [d; 0], e = [e; 0] (pn and pn - 1 entries),
//                u = [b_hat; delta] (pm), v = [c_hat; gamma] (pn);
//   flipped:     d, e reversed (r, r - 1 entries), u = [J c_hat; gamma],
//                v = J b_hat (J: reversal of r entries).
// grid (pm), up to 1024 lanes.
__global__ void track_setup_kernel(TrackMiddle mid, TrackSides s, const double *d, const double *e, int r,
                                   double delta, double gamma, double *u, double *v)
{
    const int col = blockIdx.x;
    for (int i = threadIdx.x; i < mid.pm; i += blockDim.x) {
        mid.Q[i + (int64_t)col * mid.ldq] = i == col ? 1.0 : 0.0;
        if (col < mid.pn && i < mid.pn) mid.P[i + (int64_t)col * mid.ldp] = i == col ? 1.0 : 0.0;
    }
    if (col != 0) return;
    const double *bh = s.side[0].xhat, *ch = s.side[1].xhat;
    for (int i = threadIdx.x; i < mid.pm; i += blockDim.x) {
        if (!mid.flip) {
            u[i] = i < r ? bh[i] : delta;
            if (i < mid.pn) {
                v[i] = i < r ? ch[i] : gamma;
                mid.d[i] = i < r ? d[i] : 0.0;
                if (i + 1 < mid.pn) mid.e[i] = i + 1 < r ? e[i] : 0.0;
            }
        } else {
            u[i] = i < r ? ch[r - 1 - i] : gamma;
            if (i < r) {
                v[i] = bh[r - 1 - i];
                mid.d[i] = d[r - 1 - i];
                if (i + 1 < r) mid.e[i] = e[r - 2 - i];
            }
        }
    }
}

// The tracked bidiagonal after the pass.  Both sides augmented: drop the
// row and column k of the (r+1) x (r+1) result with the smallest column
// norm (d_k^2 + e_{k-1}^2 as fma(d_k, d_k, e_{k-1} e_{k-1}); ties drop the
// highest k), with 0 joining k-1 and k+1.  Otherwise the r x r result as it
// is (reversed back when flipped) and k = -1.  One block of 256 lanes.
__global__ __launch_bounds__(256) void track_truncate_kernel(TrackMiddle mid, int r, double *d, double *e,
                                                             int *kdrop)
{
    const int t = threadIdx.x;
    if (!(mid.aug[0] && mid.aug[1])) {
        for (int j = t; j < r; j += 256) d[j] = mid.d[mid.flip ? r - 1 - j : j];
        for (int j = t; j + 1 < r; j += 256) e[j] = mid.e[mid.flip ? r - 2 - j : j];
        if (t == 0) *kdrop = -1;
        return;
    }
    // The column of least norm, as a scan from j = R - 1 down that keeps the
    // first strictly smaller value would find it: the smallest value, the
    // highest index among equal ones, NaN norms never chosen, and R - 1 when
    // its own norm is NaN (nothing compares below a NaN).  Each lane scans a
    // strided share, then a tree over the lanes with the same rule.
    __shared__ double bv[256];
    __shared__ int bk[256];
    const int R = r + 1;
    auto norm = [&](int j) {
        return j == 0 ? mid.d[0] * mid.d[0] : fma(mid.d[j], mid.d[j], mid.e[j - 1] * mid.e[j - 1]);
    };
    double best = 0.0;
    int k = -1;
    for (int j = t; j < R; j += 256) {
        const double nj = norm(j);
        if (nj == nj && (k < 0 || nj < best || (nj == best && j > k))) {
            best = nj;
            k = j;
        }
    }
    bv[t] = best;
    bk[t] = k;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
            const double ov = bv[t + w];
            const int ok = bk[t + w];
            if (ok >= 0 && (bk[t] < 0 || ov < bv[t] || (ov == bv[t] && ok > bk[t]))) {
                bv[t] = ov;
                bk[t] = ok;
            }
        }
        __syncthreads();
    }
    if (t == 0) {
        const double top = norm(R - 1);
        bk[0] = (top != top || bk[0] < 0) ? R - 1 : bk[0];
        *kdrop = bk[0];
    }
    __syncthreads();
    const int kd = bk[0];
    for (int j = t; j < R - 1; j += 256) d[j] = mid.d[j < kd ? j : j + 1];
    for (int j = t; j + 1 < R - 1; j += 256) {
        const int a = j < kd ? j : j + 1, b = j + 1 < kd ? j + 1 : j + 2;
        e[j] = b == a + 1 ? mid.e[a] : 0.0;
    }
}

// out(i, j) = sum_{l < r} A(i, l) M(rm(l), cm(j)) [+ w_i M(r, cm(j))], each
// term an fma in that order.  Not flipped: M is the middle Q for side 0 and
// P for side 1, rm(l) = l, cm(j) = j, or j + 1 from the dropped index k on,
// and w (the unit complement) only on an augmented side.  Flipped
// (U2 = U J P3 J, V2 = [V, w] diag(J,1) Q3(:, 1:r) J): M is the middle P
// for side 0 and Q for side 1, rm(l) = r - 1 - l, cm(j) = r - 1 - j, and w
// on side 1 only.
//
// Register-tiled outer products: a thread accumulates kProdRows rows (256
// apart) by kProdCols columns of out, l running in order over the whole
// sum, so every entry is still the sequential fma chain above.  The block's
// kProdCols columns of M are staged in LDS kProdChunk rows of l at a time
// and read as broadcasts; A streams once per block of kProdCols columns.
// grid (ceil(rows / (256 kProdRows)), ceil(r / kProdCols), 2 sides).
constexpr int kProdRows = 2, kProdCols = 32, kProdChunk = 64;

__global__ __launch_bounds__(256) void track_product_kernel(TrackSides s, TrackMiddle mid, const int *kdrop,
                                                            double *out0, double *out1)
{
    __shared__ double Ms[kProdChunk][kProdCols];
    const int side = blockIdx.z;
    const TrackSide &t = s.side[side];
    const int64_t rows = t.rows;
    const int64_t i0 = (int64_t)blockIdx.x * (256 * kProdRows) + threadIdx.x;
    if ((int64_t)blockIdx.x * (256 * kProdRows) >= rows) return;  // the other side has more rows
    const int r = (int)t.cols;
    const int j0 = blockIdx.y * kProdCols;
    const int k = *kdrop;
    const bool useQ = mid.flip ? side == 1 : side == 0;
    const double *Mb = useQ ? mid.Q : mid.P;
    const int64_t ldm = useQ ? mid.ldq : mid.ldp;
    const bool with_w = mid.flip ? side == 1 : mid.aug[side] != 0;
    auto colof = [&](int j) { return mid.flip ? r - 1 - j : (k >= 0 && j >= k ? j + 1 : j); };
    double acc[kProdRows][kProdCols];
#pragma unroll
    for (int q = 0; q < kProdRows; ++q)
#pragma unroll
        for (int c = 0; c < kProdCols; ++c) acc[q][c] = 0.0;
    for (int l0 = 0; l0 < r; l0 += kProdChunk) {
        __syncthreads();
        for (int x = threadIdx.x; x < kProdChunk * kProdCols; x += 256) {
            const int ll = x % kProdChunk, c = x / kProdChunk, l = l0 + ll, j = j0 + c;
            Ms[ll][c] = (l < r && j < r) ? Mb[(mid.flip ? r - 1 - l : l) + (int64_t)colof(j) * ldm] : 0.0;
        }
        __syncthreads();
        const int lend = r - l0 < kProdChunk ? r - l0 : kProdChunk;
        for (int ll = 0; ll < lend; ++ll) {
            const int64_t col = (int64_t)(l0 + ll) * t.lda;
            double a[kProdRows];
#pragma unroll
            for (int q = 0; q < kProdRows; ++q) {
                const int64_t i = i0 + 256 * q;
                a[q] = i < rows ? t.A[i + col] : 0.0;
            }
#pragma unroll
            for (int c = 0; c < kProdCols; ++c) {
                const double m = Ms[ll][c];
#pragma unroll
                for (int q = 0; q < kProdRows; ++q) acc[q][c] = fma(a[q], m, acc[q][c]);
            }
        }
    }
    double *out = side == 0 ? out0 : out1;
#pragma unroll
    for (int c = 0; c < kProdCols; ++c) {
        const int j = j0 + c;
        if (j >= r) break;
        const double mw = with_w ? Mb[r + (int64_t)colof(j) * ldm] : 0.0;
#pragma unroll
        for (int q = 0; q < kProdRows; ++q) {
            const int64_t i = i0 + 256 * q;
            if (i >= rows) continue;
            double v = acc[q][c];
            if (with_w) v = fma(t.xperp[i], mw, v);
            out[i + (int64_t)j * t.lda] = v;
        }
    }
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

hipError_t launch_track_complement(const TrackSides &s, int64_t max_rows, double *npart, double *sums,
                                   hipStream_t st)
{
    const int64_t nchunk = (max_rows + kTrackChunk - 1) / kTrackChunk;
    hipLaunchKernelGGL(track_residual_kernel, dim3((unsigned)nchunk, 2), dim3(kTrackChunk), 0, st, s, npart, nchunk);
    hipLaunchKernelGGL(track_sums_kernel, dim3(1), dim3(64), 0, st, s, (const double *)npart, nchunk, sums);
    return hipGetLastError();
}

hipError_t launch_track_accumulate(const TrackSides &s, const double *add, int64_t r, int mask, hipStream_t st)
{
    hipLaunchKernelGGL(track_accumulate_kernel, dim3((unsigned)((r + 63) / 64), 2), dim3(64), 0, st, s, add, r,
                       mask);
    return hipGetLastError();
}

hipError_t launch_track_scale(const TrackSides &s, int64_t max_rows, double delta, double gamma, hipStream_t st)
{
    hipLaunchKernelGGL(track_scale_kernel, dim3((unsigned)((max_rows + 255) / 256), 2), dim3(256), 0, st, s, delta,
                       gamma);
    return hipGetLastError();
}

hipError_t launch_track_setup(const TrackMiddle &mid, const TrackSides &s, const double *d, const double *e,
                              int64_t r, double delta, double gamma, double *u, double *v, hipStream_t st)
{
    hipLaunchKernelGGL(track_setup_kernel, dim3(mid.pm), dim3(mid.pm < 1024 ? ((mid.pm + 63) / 64) * 64 : 1024), 0,
                       st, mid, s, d, e, (int)r, delta, gamma, u, v);
    return hipGetLastError();
}

hipError_t launch_track_finish(const TrackSides &s, const TrackMiddle &mid, double *d, double *e, int *kdrop,
                               int64_t max_rows, int64_t r, double *out0, double *out1, hipStream_t st)
{
    hipLaunchKernelGGL(track_truncate_kernel, dim3(1), dim3(256), 0, st, mid, (int)r, d, e, kdrop);
    hipLaunchKernelGGL(track_product_kernel, dim3((unsigned)((max_rows + 256 * kProdRows - 1) / (256 * kProdRows)),
                                                   (unsigned)((r + kProdCols - 1) / kProdCols), 2),
                       dim3(256), 0, st, s, mid, kdrop, out0, out1);
    return hipGetLastError();
}

}  // namespace bdu
