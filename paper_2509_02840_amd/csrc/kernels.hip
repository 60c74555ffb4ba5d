// kernels.hip -- gfx950 kernels of the Givens bidiagonal update
// (Brust & Saunders, Section 3.4, Algorithm 2).  FP64 throughout.
//
//  project_kernel  u = Q^T b, v = P^T c (eq. bidiagsubproblem); one lane per
//                  output, sequential fma over the rows, 64x64 tiles staged
//                  through LDS so that global reads stay coalesced.
//  spike_kernel    m > n: the reverse-order rotations that fold u(n+1:m)
//                  into u(n+1); a dependent chain, one lane.
//  (gen_kernel, the generation of phases 1 and 2, is in gen.hip.)
//  apply_kernel    accumulates the rotation streams into Q and P
//                  (eq. bidiagplus): lanes own rows, a register window of
//                  columns slides along each block of chains, and the
//                  wavefronts of a workgroup form a pipeline that passes
//                  finished columns through LDS.
//
// Rounding: every operation is rounded on its own (-ffp-contract=off);
// fma only where written; sqrt and division are IEEE.
#include <hip/hip_runtime.h>

#include "device.h"
#include "kernels.h"
#include "primitives.h"
#include "schedule.h"

namespace bdu {

__device__ __forceinline__ BlockDesc load_block(const BlockDesc *p, int b)
{
    const CONSTANT BlockDesc *q = kptr(p) + b;
    BlockDesc d;
    d.base = q->base;
    d.lmax = q->lmax;
    d.nfront = q->nfront;
    d.phase = q->phase;
    d.off = q->off;
    d.start = q->start;
    d.pad = 0;
    return d;
}

// ---- projection ---------------------------------------------------------------

// grid (tiles, handles), 64 threads.  Tile t < ceil(m/64) projects with Q,
// the rest with P.  Lane l of tile t owns output column 64 t + l.
__global__ __launch_bounds__(64) void project_kernel(HandleDev *const *hs, Gate gate)
{
    if (gate.ranks && gate.pass >= gate.ranks[blockIdx.y]) return;
    const int pass = gate.pass;
    const CONSTANT HandleDev *h = kptr(hs[blockIdx.y]);
    const int m = h->m, n = h->n;
    const int qt = (m + 63) / 64, pt = (n + 63) / 64;
    int tile = blockIdx.x;
    if (tile >= qt + pt) return;
    const GLOBAL double *A;
    const GLOBAL double *x;
    GLOBAL double *out;
    int rows, ld;
    if (tile < qt) {
        A = gptr(h->Q); x = gptr(gate.xb ? gate.xb : h->bst) + (int64_t)pass * m; out = gptr(h->u); rows = m;
        ld = h->ldq;
    } else {
        tile -= qt;
        A = gptr(h->P); x = gptr(gate.xc ? gate.xc : h->cst) + (int64_t)pass * n; out = gptr(h->v); rows = n;
        ld = h->ldp;
    }
    const int cols = rows;
    __shared__ double tileA[64 * 65];
    __shared__ double xs[64];
    const int lane = threadIdx.x;
    const int col0 = tile * 64;
    double acc = 0.0;
    for (int j0 = 0; j0 < rows; j0 += 64) {
        const int jn = rows - j0 < 64 ? rows - j0 : 64;
        // coalesced: lane reads row j0+lane of each of the tile's 64 columns
        // (rows past the end are padding inside the leading dimension)
#pragma unroll 16
        for (int c = 0; c < 64; ++c) {
            const int col = col0 + c < cols ? col0 + c : cols - 1;
            tileA[c * 65 + lane] = A[(int64_t)col * ld + j0 + lane];
        }
        xs[lane] = lane < jn ? x[j0 + lane] : 0.0;
        __syncthreads();
        for (int j = 0; j < jn; ++j) acc = fma(tileA[lane * 65 + j], xs[j], acc);
        __syncthreads();
    }
    if (col0 + lane < cols) out[col0 + lane] = acc;
}

// ---- spike (m > n) -----------------------------------------------------------------

// grid (handles), 64 threads.  For j = m..n+2 the pair (u_{j-1}, u_j) is
// rotated onto u_{j-1} (mode 2).  Rows n+1.. of the band are zero, so only u
// and the rotation list change.
__global__ __launch_bounds__(64) void spike_kernel(HandleDev *const *hs, Gate gate)
{
    if (gate.ranks && gate.pass >= gate.ranks[blockIdx.x]) return;
    const CONSTANT HandleDev *h = kptr(hs[blockIdx.x]);
    if (h->m <= h->n) return;
    const int m = h->m, n = h->n;
    __shared__ double chunk[64];
    double *u = h->u;
    double surv = u[m - 1];  // u_m
    int j = m;               // next pair is (u_{j-1}, u_j)
    while (j >= n + 2) {
        const int lo = (j - 64 > n + 1) ? j - 64 : n + 1;  // 1-based u indices lo..j-1
        const int cnt = j - lo;
        if ((int)threadIdx.x < cnt) chunk[threadIdx.x] = u[lo - 1 + threadIdx.x];
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int q = cnt - 1; q >= 0; --q) {  // pair (u_{lo+q}, u_{lo+q+1})
                double c, s, r;
                givens(chunk[q], surv, 2, c, s, r);
                h->csSp[m - (lo + q + 1)] = make_double2(c, s);
                chunk[q] = r;
                surv = r;
            }
        }
        __syncthreads();
        j = lo;
    }
    if (threadIdx.x == 0) {
        u[n] = surv;  // u_{n+1}
        for (int i = n + 1; i < m; ++i) u[i] = 0.0;
    }
}

// ---- application ----------------------------------------------------------------

__host__ __device__ constexpr int pmod(int a, int b) { return ((a % b) + b) % b; }

// Columns in the LDS ring between two wavefronts: at most 14 columns are live
// (written but not yet read), and 3 r with r | (K0 + 3) keeps slots static.
__host__ __device__ constexpr int ring_cols(int K0)
{
    int U = K0 + 3, r = 5;
    while (U % r) ++r;
    return 3 * r;
}

// Sweep one block of K = K0*NW chains over this workgroup's 64*R rows (lane l
// owns rows l, l+64, ..., l+64(R-1) of the panel).  Wavefront w holds local
// columns [3(f-K0+1), 3f+9] of its rows in registers (f = its local front),
// applies chains w*K0 .. w*K0+K0-1 at each front, and hands finished columns
// to wavefront w+1 through an LDS ring (the last wavefront writes them back to
// memory).  Every front of the loop has a slot per chain (identity where the
// chain has no rotation), so the body has no data-dependent branches around
// the rotations.  Columns outside the block are loaded from a clamped address
// and never stored: an identity rotation leaves a finite partner unchanged,
// and real rotations never touch them.  Each coefficient pair serves R rows.
template <int K0, int NW, int R, int MODE>
__device__ __forceinline__ void sweep(GLOBAL double *__restrict__ X, int ld, int ncols, int row0,
                                      const CONSTANT double *__restrict__ cs, const BlockDesc bd,
                                      double *ring, int w, int lane)
{
    constexpr int U = K0 + 3, WSZ = 3 * U, S = U, K = K0 * NW;
    constexpr bool DESC = MODE < 2;
    constexpr int DIR = DESC ? -1 : 1;
    const int lmax = bd.lmax;
    if (lmax < 0) return;
    const int nfront = bd.nfront;
    const int base = bd.base;
    // local columns lam in [lam_lo, lam_hi] exist in this block and matrix
    const int lam_hi = lmax + 1;
    const int lam_lo = DESC ? (base - ncols > 0 ? base - ncols : 0) : 0;
    const int col0 = base - 1;  // 0-based matrix column of local column 0
    double buf[R][WSZ];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int i = 0; i < WSZ; ++i) buf[r][i] = 0.0;

    // column base address is uniform; the lane adds its row
    auto colptr = [&](int lam) -> const GLOBAL double * {
        int c = col0 + DIR * lam;
        c = c < 0 ? 0 : (c >= ncols ? ncols - 1 : c);
        return X + (int64_t)c * ld;
    };
    // ring slot of local column lam is lam mod RC (RC = ring_cols(K0) divides
    // WSZ, so the slot is a compile-time constant in the unrolled loop)
    constexpr int RC = ring_cols(K0);
    double *rin = ring + (w > 0 ? w - 1 : 0) * RC * 64 * R + lane;
    double *rout = ring + w * RC * 64 * R + lane;

    if (w == 0) {
#pragma unroll
        for (int k = 0; k <= 6; ++k) {
            const GLOBAL double *cp = colptr(k);
#pragma unroll
            for (int r = 0; r < R; ++r) buf[r][k] = cp[row0 + 64 * r];
        }
    }
    // Coefficients come in groups of G rotations.  The address of the group
    // after next (crossing into the next front at a front's end) is made
    // opaque two groups early, so its scalar loads are issued while the
    // current group computes but are never hoisted further (scalar registers
    // are few).
    constexpr int G = K0 % 4 == 0 ? 4 : 3;
    constexpr int NG = K0 / G;
    static_assert(K0 % G == 0 && NG >= 2 && K0 <= 24, "coefficient groups must tile a front");
    constexpr FrontOrder ord = front_order(MODE, K, K0);
    // Chunks of U = S fronts where this wavefront meets only identity
    // rotations (pipeline fill, local fronts f < 0; drain, after its last
    // column has left the window) only keep the workgroup's barriers.
    // Live chunks are F0 = w S + c U, c = 0 .. ceil((flush_end + 1) / U) - 1.
    const int flush_end = lam_hi / 3 + K0 - 1;
    const int nchunk = nfront / U;
    int live_end = w + (flush_end + U) / U;  // one past the last live chunk
    live_end = live_end < nchunk ? live_end : nchunk;
    auto idle = [&](int chunks) {
        if (NW > 1)
            for (int c = 0; c < chunks * U; ++c) __syncthreads();
    };
    idle(w);
    for (int F0 = w * S; F0 < live_end * U; F0 += U) {
        const CONSTANT double *pg = cs + 2 * ((int64_t)F0 * K + w * K0);
        const CONSTANT double *pg1 = pg + 2 * G;  // always two groups in flight
        asm volatile("" : "+s"(pg));
        asm volatile("" : "+s"(pg1));
#pragma unroll
        for (int phi = 0; phi < U; ++phi) {
            const int F = F0 + phi;
            const int f = F - w * S;
            // new columns: from memory (first wavefront, two fronts ahead) or
            // from the previous wavefront's ring
            if (w == 0) {
#pragma unroll
                for (int k = 7; k <= 9; ++k) {
                    const GLOBAL double *cp = colptr(3 * f + k);
#pragma unroll
                    for (int r = 0; r < R; ++r) buf[r][pmod(3 * phi + k, WSZ)] = cp[row0 + 64 * r];
                }
            } else {
                if (phi == 0 && f == 0) {
#pragma unroll
                    for (int r = 0; r < R; ++r) buf[r][0] = rin[64 * r];
                }
#pragma unroll
                for (int k = 1; k <= 3; ++k)
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        buf[r][pmod(3 * phi + k, WSZ)] = rin[(pmod(3 * phi + k, RC) * R + r) * 64];
            }
            // this wavefront's K0 rotations at front F, in front_order (their
            // coefficients are stored in that order)
            const CONSTANT double *csF = cs + 2 * ((int64_t)F * K + w * K0);
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                // address of the group after next (crossing into the next front)
                const int gg = g + 2;
                const CONSTANT double *pn = csF + (gg < NG ? 2 * G * gg : 2 * K + 2 * G * (gg - NG));
                asm volatile("" : "+s"(pn));
#pragma unroll
                for (int q = 0; q < G; ++q) {
                    const int t = ord.t[g * G + q];
                    const int l0 = 3 * (phi - t) + rho_of(MODE, K, t);
                    const int sx = pmod(l0 + (DESC ? 1 : 0), WSZ);
                    const int sy = pmod(l0 + (DESC ? 0 : 1), WSZ);
                    const double c = pg[2 * q], sn = pg[2 * q + 1];
#pragma unroll
                    for (int r = 0; r < R; ++r) rot(c, sn, buf[r][sx], buf[r][sy]);
                }
                pg = pg1;
                pg1 = pn;
            }
            // finished columns leave the window
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int lam = 3 * (f - K0 + 1) + k;
                const int sl = pmod(3 * (phi - K0 + 1) + k, WSZ);
                if (w == NW - 1) {
                    if (lam >= lam_lo && lam <= lam_hi) {
                        GLOBAL double *cp = X + (int64_t)(col0 + DIR * lam) * ld;
#pragma unroll
                        for (int r = 0; r < R; ++r) cp[row0 + 64 * r] = buf[r][sl];
                    }
                } else {
#pragma unroll
                    for (int r = 0; r < R; ++r) rout[(pmod(3 * (phi - K0 + 1) + k, RC) * R + r) * 64] = buf[r][sl];
                }
            }
            if (NW > 1) __syncthreads();
            // keep fronts in order: the columns in use (local 3(f-K0+1) ..
            // 3f+3) are materialised here, so the scheduler cannot interleave
            // two fronts (and their coefficients).  Columns loaded ahead are
            // left out: their loads stay in flight until first use.
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int j = -3 * (K0 - 1); j <= 3; ++j) asm volatile("" : "+v"(buf[r][pmod(3 * phi + j, WSZ)]));
        }
    }
    idle(nchunk - (live_end > w ? live_end : w));
}

// Spike rotations on Q columns (j-1, j), j = m..n+2, for one row: a running
// carry keeps column j between consecutive rotations.
__device__ void spike_apply(GLOBAL double *Q, int ld, int m, int n, int row, const CONSTANT double *cs)
{
    double carry = Q[(int64_t)(m - 1) * ld + row];
    for (int t = 0; t < m - n - 1; ++t) {
        const int xc = m - 2 - t;  // 0-based column of the pair's first entry
        double x = Q[(int64_t)xc * ld + row];
        rot(cs[2 * t], cs[2 * t + 1], x, carry);
        Q[(int64_t)(xc + 1) * ld + row] = carry;
        carry = x;
    }
    Q[(int64_t)n * ld + row] = carry;
}

// grid (panels, handles): panels [0, ceil(m/(64R))) update Q, the rest P.  Q
// and P have leading dimensions padded to a multiple of 128 rows.
//
// Occupancy: at one wavefront per SIMD a rotation loop issues at well under
// half the FP64 rate, so the register budget is capped to keep at least two
// wavefronts per SIMD (the (12, *, 2) tilings fit 256 registers without
// spilling; the smaller windows fit three).
template <int K0, int NW, int R>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(K0 * R >= 24 ? 2 : 3))) void apply_kernel(
    HandleDev *const *hs, Gate gate)
{
    // Workgroups are dispatched round-robin over the 8 XCDs.  Renumber them so
    // that the panels of one handle run on the same XCD and share its L2 copy
    // of the handle's rotation streams.
    const int total = gridDim.x * gridDim.y;
    const int lin = blockIdx.y * gridDim.x + blockIdx.x;
    int item = lin;
    if (total % 8 == 0) item = (lin % 8) * (total / 8) + lin / 8;
    const int hidx = item / gridDim.x, pid = item % gridDim.x;
    if (gate.ranks && gate.pass >= gate.ranks[hidx]) return;
    const CONSTANT HandleDev *h = kptr(hs[hidx]);
    const int m = h->m, n = h->n;
    constexpr int PH = 64 * R;
    const int qp = (m + PH - 1) / PH, pp = (n + PH - 1) / PH;
    if (pid >= qp + pp) return;
    constexpr int RING = (NW > 1 ? NW - 1 : 1) * ring_cols(K0) * 64 * R;
    __shared__ double ring[RING];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    // the ring starts finite (stale slots may meet identity rotations)
    for (int i = threadIdx.x; i < RING; i += 64 * NW) ring[i] = 0.0;
    const int nb1 = h->nb1;
    // blocks of this part (phase 1 = [0, nb1), phase 2 = [nb1, nb1 + nb2))
    int bbeg, bend;
    const bool spike_part = part_blocks(h, gate.part, &bbeg, &bend);
    const int b1a = bbeg < nb1 ? bbeg : nb1, b1e = bend < nb1 ? bend : nb1;  // phase-1 blocks [b1a, b1e)
    const int b2a = bbeg > nb1 ? bbeg : nb1, b2e = bend;                     // phase-2 blocks [b2a, b2e)
    if (pid < qp) {
        const int row0 = pid * PH + lane;
        GLOBAL double *Q = gptr(h->Q);
        if (m > n && w == 0 && spike_part) {
#pragma unroll
            for (int r = 0; r < R; ++r) spike_apply(Q, h->ldq, m, n, row0 + 64 * r, kptr((const double *)h->csSp));
        }
        __syncthreads();
        for (int b = b1a; b < b1e; ++b) {
            const BlockDesc bd = load_block(h->blkL, b);
            sweep<K0, NW, R, 0>(Q, h->ldq, m, row0, kptr((const double *)h->csL) + 2 * bd.off, bd, ring, w, lane);
            __syncthreads();
        }
        for (int b = b2a; b < b2e; ++b) {
            const BlockDesc bd = load_block(h->blkL, b);
            sweep<K0, NW, R, 2>(Q, h->ldq, m, row0, kptr((const double *)h->csL) + 2 * bd.off, bd, ring, w, lane);
            __syncthreads();
        }
    } else {
        const int row0 = (pid - qp) * PH + lane;
        GLOBAL double *P = gptr(h->P);
        for (int b = b1a; b < b1e; ++b) {
            const BlockDesc bd = load_block(h->blkR, b);
            sweep<K0, NW, R, 1>(P, h->ldp, n, row0, kptr((const double *)h->csR) + 2 * bd.off, bd, ring, w, lane);
            __syncthreads();
        }
        for (int b = b2a; b < b2e; ++b) {
            const BlockDesc bd = load_block(h->blkR, b);
            sweep<K0, NW, R, 3>(P, h->ldp, n, row0, kptr((const double *)h->csR) + 2 * bd.off, bd, ring, w, lane);
            __syncthreads();
        }
    }
}

// ---- staged application ---------------------------------------------------------
//
// A workgroup of NW compute wavefronts and one memory wavefront (index NW).
// The compute wavefronts run the register-window sweep above with their
// column traffic through LDS only: wavefront w takes its new columns from
// ring w and hands its finished columns to ring w + 1.  The memory wavefront
// feeds ring 0 from global memory, DL fronts ahead, and writes the columns
// arriving in ring NW back to Q or P, so no compute wavefront issues a
// global load or store.
//
// Coefficient delivery.  A (c, s) pair is uniform across the rows, so the
// compute wavefronts hold it in scalar registers, loaded from the rotation
// stream by scalar loads (sweep_compute_sc), and a rotation is four FP64
// instructions with scalar operands.  A broadcast LDS read per rotation
// would move 1 KB through the LDS data path for 16 bytes of data (the LDS
// then bounds the kernel), and a row broadcast by DPP moves costs two more
// vector instructions per rotation.  The memory wavefront touches every
// 128-byte line of a front's coefficients a few fronts ahead (one load per
// line, its value unused), which brings them into the L2 cache for the
// compute wavefronts' scalar loads; without it the scalar loads miss to
// HBM and the applier runs at half the speed.
template <int K0, int NW, int R>
struct Staged {
    static constexpr int U = K0 + 3, WSZ = 3 * U, S = U, K = K0 * NW;
    static constexpr int RC = ring_cols(K0);
    static constexpr int RING = RC * 64 * R;                  // doubles per ring
    static constexpr int LDS_DOUBLES = (NW + 1) * RING;       // rings 0 .. NW
    static constexpr int DL = U / 3;                          // memory prefetch depth, U % DL == 0
    static constexpr int NPF = (2 * K + 15) / 16 + 1;         // 128-byte lines of a front's pairs, at most
    static_assert(U % 3 == 0 && U % DL == 0 && (3 * U) % RC == 0, "static ring slots");
};

// Rotations at positions [P, P1) of a front in front_order, pair p's
// coefficients in (c[p], s[p]).
template <int K0, int R, int MODE, int K, int WSZ, int P, int P1>
__device__ __forceinline__ void front_part(const double (&c)[K0], const double (&s)[K0], double (&buf)[R][WSZ],
                                           int phi)
{
    if constexpr (P < P1) {
        constexpr FrontOrder ord = front_order(MODE, K, K0);
        constexpr bool DESC = MODE < 2;
        constexpr int t = ord.t[P];
        const int l0 = 3 * (phi - t) + rho_of(MODE, K, t);
        const int sx = pmod(l0 + (DESC ? 1 : 0), WSZ);
        const int sy = pmod(l0 + (DESC ? 0 : 1), WSZ);
#pragma unroll
        for (int r = 0; r < R; ++r) rot(c[P], s[P], buf[r][sx], buf[r][sy]);
        front_part<K0, R, MODE, K, WSZ, P + 1, P1>(c, s, buf, phi);
    }
}

// Compute wavefronts with their coefficients in scalar registers (scalar
// loads from the rotation stream): pair p of front F sits at
// cs[2 (F K + w K0 + p)].  The first half of a front's pairs is loaded in
// the middle of the previous front (once the first half of its rotations
// has freed those registers), the second half at the start of the front
// itself, so every scalar load has about half a front of work before its
// value is needed.  Scalar loads share their completion counter with LDS
// accesses and complete out of order, so every wait for one is a wait for
// all: the front's LDS accesses are all issued before the mid-front wait,
// and the barrier that ends the front waits for nothing more (a
// __syncthreads would also wait for the next front's first-half loads just
// issued; they are waited for after the barrier, before the second half's
// loads go out).
//
// One block's live chunks for compute wavefront w: nlive chunks of U fronts
// from the block's front w S (the caller has run the barriers before it).
template <int K0, int NW, int R, int MODE>
__device__ __forceinline__ void sweep_compute_sc(const CONSTANT double *__restrict__ cs, double *lds, int w, int lane,
                                                 int nlive)
{
    using T = Staged<K0, NW, R>;
    constexpr int U = T::U, WSZ = T::WSZ, S = T::S, K = T::K, RC = T::RC;
    constexpr int H = K0 / 2;
    double buf[R][WSZ];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int i = 0; i < WSZ; ++i) buf[r][i] = 0.0;
    const double *rin = lds + w * T::RING + lane;
    double *rout = lds + (w + 1) * T::RING + lane;
    const int live_end = w + nlive;
    double c[K0], sn[K0];
    // pairs [p0, p1) of front F
    auto load = [&](int F, int p0, int p1) {
        const CONSTANT double *q = cs + 2 * ((int64_t)F * K + w * K0);
#pragma unroll
        for (int p = 0; p < K0; ++p)
            if (p >= p0 && p < p1) {
                c[p] = q[2 * p];
                sn[p] = q[2 * p + 1];
            }
    };
    load(w * S, 0, H);
    for (int F0 = w * S; F0 < live_end * U; F0 += U) {
#pragma unroll
        for (int phi = 0; phi < U; ++phi) {
            const int F = F0 + phi;
            const int f = F - w * S;
            // the first half's pairs (loaded during the previous front) have
            // landed before the second half's loads are issued
            asm volatile("" ::"s"(c[0]));
            __builtin_amdgcn_sched_barrier(0);
            load(F, H, K0);
            __builtin_amdgcn_sched_barrier(0);
            if (phi == 0 && f == 0) {
#pragma unroll
                for (int k = 0; k <= 3; ++k)
#pragma unroll
                    for (int r = 0; r < R; ++r) buf[r][k] = rin[(k * R + r) * 64];
            }
            // the next front's new columns 3f+4 .. 3f+6, read a front early:
            // their producer finished them two fronts ago, and their slots
            // are not pinned, so the reads complete during this front
#pragma unroll
            for (int k = 4; k <= 6; ++k)
#pragma unroll
                for (int r = 0; r < R; ++r)
                    buf[r][pmod(3 * phi + k, WSZ)] = rin[(pmod(3 * phi + k, RC) * R + r) * 64];
            // this wavefront's K0 rotations at front F, in front_order (their
            // coefficients are stored in that order); the first ones (chain
            // K0 - 1) finish the columns that leave the window
            front_part<K0, R, MODE, K, WSZ, 0, H>(c, sn, buf, phi);
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int r = 0; r < R; ++r)
                    rout[(pmod(3 * (phi - K0 + 1) + k, RC) * R + r) * 64] = buf[r][pmod(3 * (phi - K0 + 1) + k, WSZ)];
            // wait here (not after the next loads) for this front's second
            // half: a wait for one scalar load waits for all in flight
            // every LDS access of this front (the column reads and writes
            // above) is complete after this wait
            asm volatile("" ::"s"(c[H]));
            asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
            __builtin_amdgcn_sched_barrier(0);
            load(F + 1, 0, H);
            __builtin_amdgcn_sched_barrier(0);
            front_part<K0, R, MODE, K, WSZ, H, K0>(c, sn, buf, phi);
            asm volatile("s_barrier" ::: "memory");
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int j = -3 * (K0 - 1); j <= 3; ++j) asm volatile("" : "+v"(buf[r][pmod(3 * phi + j, WSZ)]));
        }
    }
}

// A block as the memory wavefront sees it.
struct MemBlock {
    int rel;           // first chunk, relative to the launch's first block
    int nfront, C;     // fronts of the block; live chunks of each compute wavefront
    int dir, col0;     // matrix column of local column lam: col0 + dir lam
    int lam_lo, lam_hi;
    int64_t off;       // first slot of the block's pairs
};

__device__ __forceinline__ MemBlock mem_block(const BlockDesc &bd, int start0, int ncols, int K0, int U)
{
    MemBlock v;
    const bool desc = bd.phase == 1;
    v.rel = bd.start - start0;
    v.nfront = bd.nfront;
    v.lam_hi = bd.lmax + 1;
    v.C = (v.lam_hi / 3 + K0 - 1 + U) / U;
    v.dir = desc ? -1 : 1;
    v.col0 = bd.base - 1;
    v.lam_lo = desc ? (bd.base - ncols > 0 ? bd.base - ncols : 0) : 0;
    v.off = bd.off;
    return v;
}

// First block at or after b with work (lmax >= 0), or bend.
__device__ __forceinline__ int next_block(const BlockDesc *blk, int b, int bend)
{
    while (b < bend && load_block(blk, b).lmax < 0) ++b;
    return b;
}

// The memory wavefront over all blocks [bbeg, bend) of a launch, which run
// back to back (start chunks from the plan): T chunks of U fronts, one
// barrier per front.  Its load side follows the block of its latest
// prologue (the block compute wavefront 0 is in or waits for): at front F
// of that block it writes to ring 0 the columns wavefront 0 reads at front
// F + 1 (3F + 7 .. 3F + 9, loaded DL fronts earlier into a register FIFO);
// a block's columns 0..6 and first DL FIFO entries are loaded in its
// prologue, the front before it starts, which also overwrites whatever the
// load side wrote for the previous block past its end.  Its store side
// follows the oldest block not yet written back: at front F it stores the
// columns the last compute wavefront finished at front F - 1.  Every front
// it also touches every 128-byte line of the pairs the compute wavefronts
// of the load block, of the block before it and of the store block read
// DL + 2 fronts later (one word per line, its value unused), which brings
// them into the L2 cache for their scalar loads.  All its loads are issued
// at every front, whether or not their data is needed, so that the
// compiler can count them and wait only for the FIFO entry in use.  A
// column is loaded for one block only after an earlier block's store of it
// has completed; the plan's start chunks guarantee that (stage_starts in
// plan.cpp).
template <int K0, int NW, int R>
__device__ __forceinline__ void memory_wavefront(GLOBAL double *__restrict__ X, int ld, int ncols, int row0,
                                                 const CONSTANT double *cs, const BlockDesc *blk, int bbeg,
                                                 int bend, int start0, int T, double *lds, int lane)
{
    using TS = Staged<K0, NW, R>;
    constexpr int U = TS::U, S = TS::S, K = TS::K, RC = TS::RC, DL = TS::DL, NPF = TS::NPF;
    double *rw = lds + lane;                          // ring 0
    const double *rr = lds + NW * TS::RING + lane;    // ring NW
    const GLOBAL double *cg = (const GLOBAL double *)(uintptr_t)cs;
    auto colptr = [&](const MemBlock &v, int lam) -> const GLOBAL double * {
        int c = v.col0 + v.dir * lam;
        c = c < 0 ? 0 : (c >= ncols ? ncols - 1 : c);
        return X + (int64_t)c * ld;
    };
    // one word of every 128-byte line of front Fc's pairs (lanes below NPF;
    // the others load the last word again, so that the load is not under a
    // branch and the compiler can count it)
    const int q_touch = 16 * lane < 2 * K && lane < NPF ? 16 * lane : 2 * K - 1;
    auto touch = [&](const MemBlock &v, int Fc) -> double {
        Fc = Fc < 0 ? 0 : (Fc < v.nfront ? Fc : v.nfront - 1);
        return cg[2 * (v.off + (int64_t)Fc * K) + q_touch];
    };
    const int bfirst = next_block(blk, bbeg, bend);
    if (bfirst >= bend) {
        __syncthreads();
        return;  // no work: T is 0
    }
    // FIFO entry for front Fl of the load block (written to LDS at front
    // Fl): the columns 3 Fl + 7 .. 3 Fl + 9 wavefront 0 reads at front
    // Fl + 1, and the touch of its front Fl + 2
    double colf[DL][3][R];
    double pfl[DL], pfp[DL], pfs[DL];
#pragma unroll
    for (int j = 0; j < DL; ++j) pfl[j] = pfp[j] = pfs[j] = 0.0;
    MemBlock L = mem_block(load_block(blk, bfirst), start0, ncols, K0, U);
    MemBlock Pv = L, St = L;  // the block before the load block; the store block
    auto load_entry = [&](int slot, int Fl) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const GLOBAL double *cp = colptr(L, 3 * Fl + 7 + k);
#pragma unroll
            for (int r = 0; r < R; ++r) colf[slot][k][r] = cp[row0 + 64 * r];
        }
        pfl[slot] = touch(L, Fl + 2);
    };
    auto prologue = [&]() {
#pragma unroll
        for (int k = 0; k <= 6; ++k) {
            const GLOBAL double *cp = colptr(L, k);
#pragma unroll
            for (int r = 0; r < R; ++r) rw[(k * R + r) * 64] = cp[row0 + 64 * r];
        }
#pragma unroll
        for (int j = 0; j < DL; ++j) {
            asm volatile("" ::"v"(pfl[j]));
            load_entry(j, j);
        }
    };
    prologue();
    int bs = bfirst;                               // store block
    int bn = next_block(blk, bfirst + 1, bend);    // next block to load
    int next_pro = bn < bend ? mem_block(load_block(blk, bn), start0, ncols, K0, U).rel * U - 1 : -2;
    __syncthreads();
    for (int G0 = 0; G0 < T * U; G0 += U) {
#pragma unroll
        for (int phi = 0; phi < U; ++phi) {
            const int G = G0 + phi;
            const int slot = phi % DL;
            // load side (past the block's end it feeds nobody; the next
            // prologue overwrites those slots)
            {
                const int Fl = G - L.rel * U;
#pragma unroll
                for (int k = 0; k < 3; ++k)
#pragma unroll
                    for (int r = 0; r < R; ++r) rw[(pmod(3 * phi + 7 + k, RC) * R + r) * 64] = colf[slot][k][r];
                asm volatile("" ::"v"(pfl[slot]));
                load_entry(slot, Fl + DL);
                asm volatile("" ::"v"(pfp[slot]));
                pfp[slot] = touch(Pv, G - Pv.rel * U + DL + 2);
            }
            // store side
            {
                const int Fs = G - St.rel * U;
                asm volatile("" ::"v"(pfs[slot]));
                pfs[slot] = touch(St, Fs + DL + 2);
                double outv[3][R];
#pragma unroll
                for (int k = 0; k < 3; ++k)
#pragma unroll
                    for (int r = 0; r < R; ++r) outv[k][r] = rr[(pmod(3 * phi - 3 * K0 + k, RC) * R + r) * 64];
                if (bs < bend) {
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        const int lam = 3 * (Fs - 1 - (NW - 1) * S - K0 + 1) + k;
                        if (lam >= St.lam_lo && lam <= St.lam_hi) {
                            GLOBAL double *cp = X + (int64_t)(St.col0 + St.dir * lam) * ld;
#pragma unroll
                            for (int r = 0; r < R; ++r) cp[row0 + 64 * r] = outv[k][r];
                        }
                    }
                    // the block's last column is stored at this front
                    if (Fs >= St.lam_hi / 3 + (NW - 1) * S + K0) {
                        bs = next_block(blk, bs + 1, bend);
                        if (bs < bend) St = mem_block(load_block(blk, bs), start0, ncols, K0, U);
                    }
                }
            }
            // the next block's prologue, the front before it starts (always
            // the last front of a chunk: blocks start on chunk boundaries)
            if (phi == U - 1 && G == next_pro) {
                Pv = L;
                L = mem_block(load_block(blk, bn), start0, ncols, K0, U);
                prologue();
                bn = next_block(blk, bn + 1, bend);
                next_pro = bn < bend ? mem_block(load_block(blk, bn), start0, ncols, K0, U).rel * U - 1 : -2;
            }
            __syncthreads();
        }
    }
}

template <int K0, int NW, int R>
__global__ __launch_bounds__(64 * (NW + 1)) __attribute__((amdgpu_waves_per_eu(R == 2 || K0 > 12 ? 2 : 4)))
void apply_staged_kernel(HandleDev *const *hs, Gate gate)
{
    using T = Staged<K0, NW, R>;
    const int total = gridDim.x * gridDim.y;
    const int lin = blockIdx.y * gridDim.x + blockIdx.x;
    int item = lin;
    if (total % 8 == 0) item = (lin % 8) * (total / 8) + lin / 8;
    const int hidx = item / gridDim.x, pid = item % gridDim.x;
    if (gate.ranks && gate.pass >= gate.ranks[hidx]) return;
    const CONSTANT HandleDev *h = kptr(hs[hidx]);
    const int m = h->m, n = h->n;
    constexpr int PH = 64 * R;
    const int qp = (m + PH - 1) / PH, pp = (n + PH - 1) / PH;
    if (pid >= qp + pp) return;
    __shared__ double lds[T::LDS_DOUBLES];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    for (int i = threadIdx.x; i < T::LDS_DOUBLES; i += 64 * (NW + 1)) lds[i] = 0.0;
    const int nb1 = h->nb1;
    const bool onQ = pid < qp;
    const int row0 = (onQ ? pid : pid - qp) * PH + lane;
    GLOBAL double *X = gptr(onQ ? h->Q : h->P);
    const int ld = onQ ? h->ldq : h->ldp;
    const int ncols = onQ ? m : n;
    const BlockDesc *blk = onQ ? h->blkL : h->blkR;
    const CONSTANT double *cs = kptr((const double *)(onQ ? h->csL : h->csR));
    int bbeg, bend;
    const bool spike_part = part_blocks(h, gate.part, &bbeg, &bend);
    if (onQ && m > n && w == 0 && spike_part) {
#pragma unroll
        for (int r = 0; r < R; ++r) spike_apply(X, ld, m, n, row0 + 64 * r, kptr((const double *)h->csSp));
    }
    __syncthreads();
    // The launch's blocks run back to back from their planned start chunks
    // (chunks of U fronts, relative to the first block): T chunks in all,
    // the last ending when the latest block's last column is stored.  Every
    // wavefront runs one barrier after the memory wavefront's first
    // prologue and one per front of the T chunks.
    constexpr int U = T::U;
    const int start0 = bbeg < bend ? load_block(blk, bbeg).start : 0;
    int Tch = 0;
    for (int b = bbeg; b < bend; ++b) {
        const BlockDesc bd = load_block(blk, b);
        if (bd.lmax < 0) continue;
        const int e = bd.start - start0 + bd.nfront / U;
        Tch = Tch > e ? Tch : e;
    }
    if (w == NW) {
        memory_wavefront<K0, NW, R>(X, ld, ncols, row0, cs, blk, bbeg, bend, start0, Tch, lds, lane);
        return;
    }
    __syncthreads();  // the memory wavefront's first prologue is in LDS
    int cur = 0;      // chunks of barriers run so far
    for (int b = bbeg; b < bend; ++b) {
        const BlockDesc bd = load_block(blk, b);
        if (bd.lmax < 0) continue;
        const int rel = bd.start - start0;
        const int C = ((bd.lmax + 1) / 3 + K0 - 1 + U) / U;
        const int nc = bd.nfront / U - w;
        const int nlive = C < nc ? C : nc;
        for (int i = (rel + w - cur) * U; i > 0; --i) __syncthreads();
        cur = rel + w + nlive;
        const CONSTANT double *cb = cs + 2 * bd.off;
        if (b < nb1) {
            if (onQ) sweep_compute_sc<K0, NW, R, 0>(cb, lds, w, lane, nlive);
            else sweep_compute_sc<K0, NW, R, 1>(cb, lds, w, lane, nlive);
        } else {
            if (onQ) sweep_compute_sc<K0, NW, R, 2>(cb, lds, w, lane, nlive);
            else sweep_compute_sc<K0, NW, R, 3>(cb, lds, w, lane, nlive);
        }
    }
    for (int i = (Tch - cur) * U; i > 0; --i) __syncthreads();
}

// The rotation primitive on arrays (checks the device arithmetic against the
// reference bit for bit).
__global__ void givens_kernel(const double *a, const double *b, int mode, double *c, double *s, double *r,
                              int64_t count)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        double cc, ss, rr;
        givens(a[i], b[i], mode, cc, ss, rr);
        c[i] = cc;
        s[i] = ss;
        r[i] = rr;
    }
}

hipError_t launch_givens(const double *a, const double *b, int mode, double *c, double *s, double *r,
                         int64_t count, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(givens_kernel, dim3((unsigned)blocks), dim3(256), 0, st, a, b, mode, c, s, r, count);
    return hipGetLastError();
}

// Fill rotation streams with the identity (c, s) = (1, 0).
__global__ void fill_identity_kernel(double2 *p, int64_t count)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = make_double2(1.0, 0.0);
}

// ---- launchers ---------------------------------------------------------------------

hipError_t launch_project(HandleDev *const *hs, int count, int max_tiles, Gate gate, hipStream_t st)
{
    hipLaunchKernelGGL(project_kernel, dim3(max_tiles, count), dim3(64), 0, st, hs, gate);
    return hipGetLastError();
}

hipError_t launch_spike(HandleDev *const *hs, int count, Gate gate, hipStream_t st)
{
    hipLaunchKernelGGL(spike_kernel, dim3(count), dim3(64), 0, st, hs, gate);
    return hipGetLastError();
}

template <int K0, int NW, int R>
static hipError_t launch_apply_t(HandleDev *const *hs, int count, int max_panels, Gate gate, hipStream_t st)
{
    hipLaunchKernelGGL((apply_kernel<K0, NW, R>), dim3(max_panels, count), dim3(64 * NW), 0, st, hs, gate);
    return hipGetLastError();
}

template <int K0, int NW, int R>
static hipError_t launch_staged_t(HandleDev *const *hs, int count, int max_panels, Gate gate, hipStream_t st)
{
    hipLaunchKernelGGL((apply_staged_kernel<K0, NW, R>), dim3(max_panels, count), dim3(64 * (NW + 1)), 0, st, hs,
                       gate);
    return hipGetLastError();
}

// nw in {1, 2, 4, 8}: nw wavefronts, each loading or storing what it needs;
// nw in {3, 5, 7, 15}: the staged kernel, nw compute wavefronts and a memory
// wavefront (k0 = 12: nw in {3, 7, 15}, rpl 2 only for nw <= 7; k0 = 18:
// nw in {3, 5, 7}, rpl 1).
bool tiling_supported(int k0, int nw, int rpl)
{
    if (nw == 3 || nw == 5 || nw == 7 || nw == 15) {
        if (k0 == 12) return nw != 5 && (rpl == 1 || (rpl == 2 && nw != 15));
        return k0 == 18 && nw != 15 && rpl == 1;
    }
    if (k0 == 6 && nw == 8 && rpl == 2) return false;  // its LDS ring exceeds 160 KB
    return (k0 == 6 || k0 == 12) && (nw == 1 || nw == 2 || nw == 4 || nw == 8) && (rpl == 1 || rpl == 2);
}

hipError_t launch_apply(HandleDev *const *hs, int count, int max_panels, int k0, int nw, int rpl, Gate gate,
                        hipStream_t st)
{
#define BDU_APPLY_CASE(A, B, C) \
    if (k0 == A && nw == B && rpl == C) return launch_apply_t<A, B, C>(hs, count, max_panels, gate, st);
    BDU_APPLY_CASE(6, 1, 1) BDU_APPLY_CASE(6, 2, 1) BDU_APPLY_CASE(6, 4, 1) BDU_APPLY_CASE(6, 8, 1)
    BDU_APPLY_CASE(12, 1, 1) BDU_APPLY_CASE(12, 2, 1) BDU_APPLY_CASE(12, 4, 1) BDU_APPLY_CASE(12, 8, 1)
    BDU_APPLY_CASE(6, 1, 2) BDU_APPLY_CASE(6, 2, 2) BDU_APPLY_CASE(6, 4, 2)
    BDU_APPLY_CASE(12, 1, 2) BDU_APPLY_CASE(12, 2, 2) BDU_APPLY_CASE(12, 4, 2) BDU_APPLY_CASE(12, 8, 2)
#undef BDU_APPLY_CASE
#define BDU_STAGED_CASE(A, B, C) \
    if (k0 == A && nw == B && rpl == C) return launch_staged_t<A, B, C>(hs, count, max_panels, gate, st);
    BDU_STAGED_CASE(12, 3, 1) BDU_STAGED_CASE(12, 7, 1) BDU_STAGED_CASE(12, 15, 1)
    BDU_STAGED_CASE(12, 3, 2) BDU_STAGED_CASE(12, 7, 2)
    BDU_STAGED_CASE(18, 3, 1) BDU_STAGED_CASE(18, 5, 1) BDU_STAGED_CASE(18, 7, 1)
#undef BDU_STAGED_CASE
    return hipErrorInvalidValue;
}

// flag[0] = 1 if any of the count values is NaN or infinite (flag[0] is
// cleared by the caller; every writer stores the same value).
__global__ void nonfinite_kernel(const double *p, int64_t count, int *flag)
{
    bool bad = false;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        bad |= !isfinite(p[i]);
    if (bad) flag[0] = 1;
}

hipError_t launch_nonfinite(const double *p, int64_t count, int *flag, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(nonfinite_kernel, dim3((unsigned)blocks), dim3(256), 0, st, p, count, flag);
    return hipGetLastError();
}

hipError_t launch_fill_identity(double2 *p, int64_t count, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_identity_kernel, dim3((unsigned)blocks), dim3(256), 0, st, p, count);
    return hipGetLastError();
}

}  // namespace bdu
