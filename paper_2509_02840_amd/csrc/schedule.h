// schedule.h -- the rotation schedule of the Givens bidiagonal update
// (Brust & Saunders, Section 3.4, Algorithm 2), decoded in closed form.
//
// The rotations of one rank-1 pass form "chains": each chain starts with one
// elimination (of an entry of u = Q^T b, of v = P^T c, or of an entry of the
// band) and continues with the bulge chase that elimination causes.
//
//   phase 1, k = 1..n-1 (eliminate v and u, keep one sub- and two
//   superdiagonals):
//     P1A(k): R(k) zeroes v_k; chase up-left: L(i), R(i-1), i = k-2, k-5, ...
//     P1B(k) (k <= N-2): L(k) zeroes u_k; R(k-1) removes (k+1, k-1);
//              chase up-left from i = k-3
//   fold: u v^T now touches only (N-1, n) and (N, n)
//   phase 2, j = 1..n (band to bidiagonal):
//     P2A(j) (j+1 <= N): L(j) zeroes (j+1, j); chase down-right:
//              R(i+2), L(i+3), i = j, j+3, ...
//     P2B(j) (j+2 <= n): R(j+1) zeroes (j, j+2); L(j+2) removes (j+3, j+1);
//              chase down-right from i = j+2
//
// L(i) rotates rows i, i+1 of the band and columns i, i+1 of Q; R(j) rotates
// columns j, j+1 of the band and of P.  N = n when m = n and n + 1 when
// m > n (row n+1 holds the survivor of the spike, handled separately).
// Indices are 1-based as in the paper.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__) || defined(__HIP__)
#include <hip/hip_runtime.h>
#define BDU_HD __host__ __device__ inline
#else
#define BDU_HD inline
#endif

namespace bdu {

enum ChainType : int32_t { CH_P1A = 1, CH_P1B = 2, CH_FOLD = 3, CH_P2A = 4, CH_P2B = 5 };

// One decoded rotation.  The generating pair is either the vector pair
// (u_i, u_{i+1}) / (v_i, v_{i+1}) (gvec = 1) or two band cells
// (gr0, gc0), (gr1, gc1).  mode 1 annihilates the first entry of the pair,
// mode 2 the second.
struct Rot {
    int32_t side;  // 0 left (rows / Q), 1 right (columns / P)
    int32_t i;     // first index of the rotated pair
    int32_t gvec;
    int32_t gr0, gc0, gr1, gc1;
    int32_t mode;
};

BDU_HD Rot rot_left(int i, int r0, int c0, int r1, int c1, int mode)
{
    Rot r;
    r.side = 0; r.i = i; r.gvec = 0; r.gr0 = r0; r.gc0 = c0; r.gr1 = r1; r.gc1 = c1; r.mode = mode;
    return r;
}
BDU_HD Rot rot_right(int j, int r0, int c0, int r1, int c1, int mode)
{
    Rot r;
    r.side = 1; r.i = j; r.gvec = 0; r.gr0 = r0; r.gc0 = c0; r.gr1 = r1; r.gc1 = c1; r.mode = mode;
    return r;
}
BDU_HD Rot rot_vec(int side, int i)
{
    Rot r;
    r.side = side; r.i = i; r.gvec = 1; r.gr0 = r.gc0 = r.gr1 = r.gc1 = 0; r.mode = 1;
    return r;
}

// Step s of the up-left chase that starts with L(i0): L(i0), R(i0-1), L(i0-3), ...
BDU_HD Rot up_chase(int i0, int s)
{
    int ii = i0 - 3 * (s >> 1);
    if ((s & 1) == 0)  // L(ii) removes (ii, ii+3), survivor (ii+1, ii+3)
        return rot_left(ii, ii, ii + 3, ii + 1, ii + 3, 1);
    // R(ii-1) removes (ii+1, ii-1), survivor (ii+1, ii)
    return rot_right(ii - 1, ii + 1, ii - 1, ii + 1, ii, 1);
}

// Step s of the down-right chase after a left rotation on rows i0, i0+1:
// R(i0+2), L(i0+3), R(i0+5), ...
BDU_HD Rot down_chase(int i0, int s)
{
    int ii = i0 + 3 * (s >> 1);
    if ((s & 1) == 0)  // R(ii+2) removes (ii, ii+3), survivor (ii, ii+2)
        return rot_right(ii + 2, ii, ii + 2, ii, ii + 3, 2);
    // L(ii+3) removes (ii+4, ii+2), survivor (ii+3, ii+2)
    return rot_left(ii + 3, ii + 3, ii + 2, ii + 4, ii + 2, 2);
}

// Rotation number s of chain (type, param).
BDU_HD Rot decode(int type, int p, int s)
{
    switch (type) {
    case CH_P1A:
        if (s == 0) return rot_vec(1, p);            // R(k) zeroes v_k
        return up_chase(p - 2, s - 1);
    case CH_P1B:
        if (s == 0) return rot_vec(0, p);            // L(k) zeroes u_k
        if (s == 1) return rot_right(p - 1, p + 1, p - 1, p + 1, p, 1);
        return up_chase(p - 3, s - 2);
    case CH_P2A:
        if (s == 0) return rot_left(p, p, p, p + 1, p, 2);
        return down_chase(p, s - 1);
    default:  // CH_P2B
        if (s == 0) return rot_right(p + 1, p, p + 1, p, p + 2, 2);
        if (s == 1) return rot_left(p + 2, p + 2, p + 1, p + 3, p + 1, 2);
        return down_chase(p + 2, s - 2);
    }
}

// Number of rotations in the up-left chase starting with L(i0).
BDU_HD int len_up(int i0)
{
    if (i0 < 1) return 0;
    int nl = (i0 - 1) / 3 + 1;
    int last = i0 - 3 * (nl - 1);
    return nl + (last >= 2 ? nl : nl - 1);
}

// Number of rotations in the down-right chase after a left rotation on rows i0, i0+1.
BDU_HD int len_down(int i0, int n, int N)
{
    int cnt = 0;
    for (int i = i0; i + 3 <= n; i += 3) {
        ++cnt;
        if (i + 4 > N) break;
        ++cnt;
    }
    return cnt;
}

// Chain index within its phase (shared by the left and the right rotation
// streams): 2(k-1) for P1A(k), 2(k-1)+1 for P1B(k), likewise for phase 2.
BDU_HD int chain_in_phase(int type, int p)
{
    return 2 * (p - 1) + ((type == CH_P1B || type == CH_P2B) ? 1 : 0);
}

BDU_HD int chain_phase(int type) { return type <= CH_P1B ? 1 : 2; }

// Applier layout of one rotation stream.  The chains of a phase are cut into
// blocks of K = K0 * NW consecutive chains.  In block b the "local column"
// lambda of a matrix column c (1-based) is
//   phase 1 (chains run towards column 1): lambda = base - c, base = k0 + K/2 + 2
//   phase 2 (chains run towards column n): lambda = c - base, base = k0
// with k0 = 1 + b*K/2 the block's first step.  A rotation of chain
// t = w*K0 + tl of the block on the pair whose lower local column is lam0
// sits at front F = floor(lam0 / 3) + tl + w*S, slot F*K + w*K0 + pos(tl),
// S = K0 + 3, where pos is the chain's place in the front's processing order
// (front_order below).
BDU_HD int block_base(int phase, int b, int K)
{
    int k0 = 1 + b * (K / 2);
    return phase == 1 ? k0 + K / 2 + 2 : k0;
}

BDU_HD int lam0_of_pair(int phase, int base, int i)
{
    return phase == 1 ? base - i - 1 : i - base;
}

// Residue mod 3 of the lower local column of the pairs of chain t (block
// index; K0 a multiple of 6 makes it the same for chain t of every
// wavefront).  mode 0: phase 1 left, 1: phase 1 right, 2: phase 2 left,
// 3: phase 2 right.  At one front chain t's pair starts at local column
// 3(f - t) + rho for the wavefront-local front f.
BDU_HD constexpr int rho_of(int mode, int K, int t)
{
    int i = t >> 1, h = t & 1;
    int v = mode == 0 ? K / 2 - i + h : mode == 1 ? K / 2 + 1 - i + h : mode == 2 ? i + 2 * h : i + 2 - h;
    return ((v % 3) + 3) % 3;
}

// Chains t and t+1 touch a common column at the same front exactly when
// rho(t+1) - rho(t) = 2; then t's rotation comes first in the update order.
BDU_HD constexpr bool shares_next(int mode, int K, int t)
{
    return rho_of(mode, K, t + 1) - rho_of(mode, K, t) == 2;
}

// Processing order of a wavefront's K0 chains within one front: last chain
// first (the columns that just entered the window, used by chain 0, are
// needed last; those leaving it, touched by chain K0-1, are final first),
// except that a pair sharing a column keeps its update order.
struct FrontOrder {
    int t[24];    // chain at each position
    int pos[24];  // position of each chain
};

BDU_HD constexpr FrontOrder front_order(int mode, int K, int K0)
{
    FrontOrder o{};
    int p = 0;
    for (int t = K0 - 1; t >= 0;) {
        if (t > 0 && shares_next(mode, K, t - 1)) {
            o.t[p++] = t - 1;
            o.t[p++] = t;
            t -= 2;
        } else {
            o.t[p++] = t;
            t -= 1;
        }
    }
    for (int q = 0; q < K0; ++q) o.pos[o.t[q]] = q;
    return o;
}

// A chain's rotations alternate sides; consecutive rotations on one side
// move three columns along the chain, i.e. one front, so rotation s lands in
// slot slot[side(s)] + (s >> 1) * K of its side's stream, side(s) =
// side(0) xor (s & 1).
struct GenChain {
    int32_t type;
    int32_t param;
    int32_t len;
    int32_t tau0;     // generation tick of the chain's first rotation
    int64_t slot[2];  // slot of the chain's first left / right rotation
};

struct BlockDesc {
    int32_t base;
    int32_t lmax;    // largest lam0 of the block (-1: empty block)
    int32_t nfront;  // fronts swept (a multiple of K0 + 3), each with K slots
    int32_t phase;
    int64_t off;     // first slot of the block in the side's stream
    int32_t start;   // staged applier: the block's first chunk of K0 + 3 fronts
                     // (blocks run back to back; see stage_starts in plan.cpp)
    int32_t pad;
};

}  // namespace bdu
