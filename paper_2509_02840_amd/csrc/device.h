// device.h -- per-handle device descriptor shared by the host library and
// the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "schedule.h"

namespace bdu {

constexpr int kMaxSeg = 8;  // most phase-2 segments of a split pass

struct GenStart;

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
    const GenStart *starts; // their first two rotations decoded (in-LDS generation; else null)
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

// Rotation s of a chain as the generation kernel addresses it: the offsets
// (in doubles from the band's start) of its five window pairs (x[k], y[k])
// in the kernel's slot order and of its u or v pair, and its side.
//
// In phase 1 both chain types are the up-left chase pattern L(ii)
// [(ii,ii+3) onto (ii+1,ii+3)], R(ii-1) [(ii+1,ii-1) onto (ii+1,ii)],
// ii = i0 - 3*(ss>>1), whose first rotation eliminates an entry of v (P1A) or
// u (P1B) instead.  In phase 2 both are the down-right pattern R(ii+2)
// [(ii,ii+3) into (ii,ii+2)], L(ii+3) [(ii+4,ii+2) into (ii+3,ii+2)],
// ii = i0 + 3*(ss>>1), whose first rotation acts one column (P2A) or one row
// (P2B) further on.  A left rotation on rows (i, i+1) rotates the band pairs
// w_j in columns i-1+j, a right rotation on columns (j', j'+1) those in rows
// j'-2+j (j = 0..4, the only pairs the schedule can make nonzero), plus the
// matching u or v pair (u at uo + i + 3, v at vo + j + 3).
//
// Consecutive rotations of a chain share two window pairs: in phase 1 pairs
// w_0, w_1 of one rotation are w_3, w_4 of the next, in phase 2 the reverse.
// The window is kept in the order (w_3, w_4, w_2, w_0, w_1) in phase 1 and
// (w_0, ..., w_4) in phase 2, so slots 0 and 1 are the pairs shared with the
// previous rotation and slots 3 and 4 those shared with the next.
struct RotOff {
    int x[5], y[5];
    int vb;
    int side;  // 0 left (rows, Q), 1 right (columns, P)
};

__host__ __device__ inline RotOff rot_offsets(int type, int param, int s, int uo, int vo)
{
    const bool ph1 = type <= CH_P1B;
    const bool first = ph1 ? (type == CH_P1A) : (type == CH_P2A);
    const int ss = s + (first ? 1 : 0);
    const int odd = ss & 1;
    const int i0 = ph1 ? (first ? param + 1 : param) : (first ? param - 3 : param - 1);
    const int ii = ph1 ? i0 - 3 * (ss >> 1) : i0 + 3 * (ss >> 1);
    const int side = ph1 ? odd : 1 - odd;
    const int i = ph1 ? (odd ? ii - 1 : ii) : (odd ? ii + 3 : ii + 2);
    RotOff o;
    o.side = side;
    o.vb = (side == 0 ? uo : vo) + i + 3;
    // left: rows i, i+1 at columns i-1..i+3; right: rows i-2..i+2 at
    // columns i, i+1 (adjacent doubles)
    const int b2 = band_row(i), b3 = band_row(i + 1);
    const int rb[5] = {band_row(i - 2) + 4, band_row(i - 1) + 3, b2 + 2, b3 + 1, band_row(i + 2)};
    int wx[5], wy[5];
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        wx[j] = side == 0 ? b2 + j + 1 : rb[j];
        wy[j] = side == 0 ? b3 + j : rb[j] + 1;
    }
    const int ord1[5] = {3, 4, 2, 0, 1};
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        o.x[k] = ph1 ? wx[ord1[k]] : wx[k];
        o.y[k] = ph1 ? wy[ord1[k]] : wy[k];
    }
    return o;
}

// A chain's first two rotations as the in-LDS generation kernel starts it,
// decoded once per shape on the host: the offsets of rotation s_e (the one
// at an even tick: 1 when the chain starts at an odd tick, else 0) in the
// low 16 bits and of the other in the high 16 bits, in the order x[0..4],
// y[0..4], vb; bit 0 of sides is the side of rotation s_e, bit 1 that of the
// other.  Offsets fit in 16 bits whenever the band does in LDS; entries of
// a rotation past the chain's end are 0 and never used.
struct GenStart {
    uint32_t off[11];
    int32_t sides;
};
static_assert(sizeof(GenStart) == 48, "the generation kernel reads 12 words per chain");

}  // namespace bdu
