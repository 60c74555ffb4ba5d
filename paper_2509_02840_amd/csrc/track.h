// track.h -- device-side descriptors and launchers of the subspace-tracking
// update (Section 4).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bdu {

// Rows per chunk of the row sums (a sequential fma inside a chunk, chunk
// partials added in ascending order).
constexpr int kTrackChunk = 256;

// One side of the tracking update: the tracked basis A (rows x cols,
// column-major, leading dimension lda = rows), the vector x (rows), its
// projection xhat (cols) and the complement xperp (rows; scaled to unit
// norm in place at the end).  x may alias xperp (second pass).
struct TrackSide {
    const double *A;
    int64_t rows, cols, lda;
    const double *x;
    double *xhat, *xperp;
};
struct TrackSides {
    TrackSide side[2];  // 0: U and b, 1: V and c
};

// The middle factorization (pm x pn, pm >= pn) before its BGU pass and the
// inputs of the pass: Q = I (pm x pm), P = I (pn x pn), d, e from the
// tracked bidiagonal (reversed when flip), u (pm), v (pn).
//   aug[side]: that side is augmented (its norm is positive);
//   flip: only the right side is augmented, so the r x (r+1) middle matrix
//         runs as its transpose with rows and columns reversed.
struct TrackMiddle {
    double *Q, *P, *d, *e;
    int64_t ldq, ldp;
    int pm, pn;
    int aug[2];
    int flip;
};

// part: 2 * ceil(max_rows / kTrackChunk) * r doubles.
hipError_t launch_track_project(const TrackSides &s, int64_t max_rows, int64_t r, double *part, hipStream_t st);
// xperp = x - A xhat; sums[side] = (x^T x, xperp^T xperp) from chunk
// partials npart (2 * 2 * chunks doubles).
hipError_t launch_track_complement(const TrackSides &s, int64_t max_rows, double *npart, double *sums,
                                   hipStream_t st);
// xhat[side] += add[side] (cols entries) for the sides in mask.
hipError_t launch_track_accumulate(const TrackSides &s, const double *add, int64_t r, int mask, hipStream_t st);
hipError_t launch_track_scale(const TrackSides &s, int64_t max_rows, double delta, double gamma, hipStream_t st);
// The middle factorization reset to identities and the pass inputs u, v.
hipError_t launch_track_setup(const TrackMiddle &mid, const TrackSides &s, const double *d, const double *e,
                              int64_t r, double delta, double gamma, double *u, double *v, hipStream_t st);
// Truncation (both sides augmented) or the copy of d, e, and the thin
// products of eq. (bdlrup) into out0 (m x r) and out1 (n x r).
hipError_t launch_track_finish(const TrackSides &s, const TrackMiddle &mid, double *d, double *e, int *kdrop,
                               int64_t max_rows, int64_t r, double *out0, double *out1, hipStream_t st);

}  // namespace bdu
