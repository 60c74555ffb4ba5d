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
// column-major, leading dimension lda = rows), the new vector x (rows),
// its projection xhat (cols + 1: the last entry receives the complement's
// norm) and the complement xperp (rows; scaled to unit norm in place).
struct TrackSide {
    const double *A;
    int64_t rows, cols, lda;
    const double *x;
    double *xhat, *xperp;
};
struct TrackSides {
    TrackSide side[2];  // 0: U and b, 1: V and c
};

// The middle (R x R) factorization's device arrays.
struct TrackMiddle {
    double *Q, *P, *d, *e;
    int64_t ldq, ldp;
    int R;
};

// part: 2 * ceil(max_rows / kTrackChunk) * r doubles; npart: 2 * ceil(max_rows / kTrackChunk).
hipError_t launch_track_project(const TrackSides &s, int64_t max_rows, int64_t r, double *part, hipStream_t st);
hipError_t launch_track_complement(const TrackSides &s, int64_t max_rows, double *npart, double *norms,
                                   hipStream_t st);
hipError_t launch_track_scale(const TrackSides &s, int64_t max_rows, hipStream_t st);
hipError_t launch_track_reset(const TrackMiddle &mid, const double *d, const double *e, hipStream_t st);
hipError_t launch_track_finish(const TrackSides &s, const TrackMiddle &mid, double *d, double *e, int *kdrop,
                               int64_t max_rows, int64_t r, double *out0, double *out1, hipStream_t st);

}  // namespace bdu
