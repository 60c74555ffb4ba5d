// device.h -- per-handle device descriptor shared by the host library and
// the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "schedule.h"

namespace bdu {

constexpr int kMaxSeg = 8;  // most phase-2 segments of a split pass

// Everything a kernel needs to update one factorization A = Q Bd P^T.
// Q is m x m and P is n x n, column-major; their leading dimensions ldq, ldp
// are m and n rounded up to a multiple of 128 (the padding rows are zero).
struct HandleDev {
    double *Q, *P, *d, *e;
    double *u, *v;          // projections u = Q^T b (m), v = P^T c (n)
    double *bst, *cst;      // staged update columns: B (m x rcap), C (n x rcap)
    double2 *csL, *csR;     // left / right rotation streams in applier layout
    double2 *csSp;          // spike rotations, in order
    double *band;           // global band scratch for large n (else unused)
    const GenChain *chains; // non-empty chains, schedule order
    const BlockDesc *blkL, *blkR;
    int64_t ticks;          // generation ticks
    int32_t m, n, N, nchains, nb1, nb2;
    int32_t ldq, ldp;
    int32_t K0, NW, K, S;
    int64_t split;          // generation split tick (Plan::split)
    // segments of a pass: segment k generates ticks [tcut[k-1], tcut[k])
    // and applies blocks [bcut[k-1], bcut[k]) (phase-1 blocks, then
    // phase-2 blocks; tcut[-1] = bcut[-1] = 0); nseg == 0: no segments
    int32_t nseg;
    int32_t tcut[kMaxSeg], bcut[kMaxSeg];
    double *carry;          // register carries of chains in flight at a segment end (4 per thread)
};

// Per-launch gate of a batch in which streams take different ranks: the
// handle at position i of a launch takes part in pass `pass` only if
// pass < ranks[i] (ranks == nullptr: every handle takes part).
// part: 0 the whole pass; 1 generation up to the end of phase 1 (with the
// fold) and application of the spike and the phase-1 blocks; 2 the rest;
// 3 + k segment k (HandleDev::tcut, bcut; segment 0 also applies the spike).
struct Gate {
    const int32_t *ranks;
    int32_t pass;
    int32_t part;
    // staged update columns of a single-handle launch when not null (m x r
    // and n x r, column-major); otherwise the handle's own staging bst, cst
    const double *xb, *xc;
};

// Applier blocks [*bbeg, *bend) of a part, and whether it applies the spike.
template <typename H>
__host__ __device__ inline bool part_blocks(const H *h, int part, int *bbeg, int *bend)
{
    const int nb1 = h->nb1, nb2 = h->nb2;
    if (part >= 3) {
        const int k = part - 3;
        if (k >= h->nseg) {  // a batch runs as many segments as its largest plan has
            *bbeg = *bend = 0;
            return false;
        }
        *bbeg = k == 0 ? 0 : h->bcut[k - 1];
        *bend = h->bcut[k];
        return k == 0;
    }
    *bbeg = part == 2 ? nb1 : 0;
    *bend = part == 1 ? nb1 : nb1 + nb2;
    return part <= 1;
}

constexpr int kGenThreads = 1024;  // at n = 2048, 256 threads leave chains waiting for a free thread

// Band storage of the generation kernel: row r (1-based, -3..N+4) starts at
// band_row(r) and holds the entries in columns r-2..r+3, column c at offset
// c - r + 2.  The extra double every three rows spreads the rows that
// neighbouring lanes touch in one tick (about seven rows apart) over the LDS
// banks (with a plain stride of six they fall on a few banks), and keeps
// band_row(r + 3) = band_row(r) + 19, so a chain's addresses move by a
// constant from one step of its pattern to the next.
__host__ __device__ inline int band_row(int r)
{
    return 6 * (r + 3) + (r + 3) / 3;
}

constexpr int kBandStep3 = 19;  // band_row(r + 3) - band_row(r)

// Doubles of the band (rows -3..N+4); u (N + 8) and v (n + 8) follow.
__host__ __device__ inline int64_t band_doubles(int64_t N)
{
    return 6 * (N + 8) + (N + 8) / 3 + 2;
}

// LDS bytes the generation kernel needs for n columns and N rows.
inline int64_t gen_lds_bytes(int64_t n, int64_t N)
{
    return 8 * (band_doubles(N) + (N + 8) + (n + 8) + 2);
}

constexpr int64_t kMaxGenLds = 160 * 1024;

}  // namespace bdu
