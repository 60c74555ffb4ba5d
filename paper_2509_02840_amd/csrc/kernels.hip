// kernels.hip -- gfx950 kernels of the Givens bidiagonal update
// (Brust & Saunders, Section 3.4, Algorithm 2).  FP64 throughout.
//
//  project_kernel  u = Q^T b, v = P^T c (eq. bidiagsubproblem); one lane per
//                  output, sequential fma over the rows, 64x64 tiles staged
//                  through LDS so that global reads stay coalesced.
//  spike_kernel    m > n: the reverse-order rotations that fold u(n+1:m)
//                  into u(n+1); a dependent chain, one lane.
//  gen_kernel      generation of phases 1 and 2 on the band held in LDS (or
//                  global memory for large n): one thread per chain in
//                  flight, one rotation per tick, ticks separated by barriers.
//  apply_kernel    accumulates the rotation streams into Q and P
//                  (eq. bidiagplus): lanes own rows, a register window of
//                  columns slides along each block of chains, and the
//                  wavefronts of a workgroup form a pipeline that passes
//                  finished columns through LDS.
//
// Rounding: every operation is rounded on its own (-ffp-contract=off);
// fma only where written; sqrt and division are IEEE.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device.h"
#include "kernels.h"
#include "schedule.h"

namespace bdu {

#define GLOBAL __attribute__((address_space(1)))
#define CONSTANT __attribute__((address_space(4)))
#define LOCAL __attribute__((address_space(3)))

// Pointers read from a descriptor are generic; the kernels know which memory
// they point to.  Global pointers give global (not flat) memory instructions,
// constant pointers with a uniform index give scalar loads.
template <typename T>
__device__ __forceinline__ GLOBAL T *gptr(T *p)
{
    return (GLOBAL T *)(uintptr_t)p;
}
template <typename T>
__device__ __forceinline__ const CONSTANT T *kptr(const T *p)
{
    return (const CONSTANT T *)(uintptr_t)p;
}

__device__ __forceinline__ BlockDesc load_block(const BlockDesc *p, int b)
{
    const CONSTANT BlockDesc *q = kptr(p) + b;
    BlockDesc d;
    d.base = q->base;
    d.lmax = q->lmax;
    d.nfront = q->nfront;
    d.phase = q->phase;
    d.off = q->off;
    return d;
}

// ---- primitives (eq. giv1) -------------------------------------------------

// Rotation generator: mode 1 gives [c -s; s c][a;b] = [0;r], mode 2 gives
// [r;0]; r = +sqrt(a^2 + b^2) with an exact power-of-two scaling when the
// larger magnitude is extreme; identity when the target is already zero.
//
// Written with selects only: both the identity and the general result are
// computed (the general one may be NaN when a = b = 0 and is then discarded),
// so a wavefront runs one straight sequence whatever its lanes' data.
template <int MODE>
__device__ __forceinline__ void givens_m(double a, double b, double &c, double &s, double &r)
{
    constexpr bool m1 = MODE == 1;
    const double fa = fabs(a), fb = fabs(b);
    const double big = fa > fb ? fa : fb;
    const bool hi = big > 0x1p500, lo = big < 0x1p-500;
    const double sc = hi ? 0x1p-600 : (lo ? 0x1p600 : 1.0);
    const double unsc = hi ? 0x1p600 : (lo ? 0x1p-600 : 1.0);
    const double as = a * sc, bs = b * sc;
    const double rs = sqrt(fma(as, as, bs * bs));
    const double p = (m1 ? bs : as) / rs, q = (m1 ? as : bs) / rs;
    const bool ident = (m1 ? a : b) == 0.0;
    c = ident ? 1.0 : p;
    s = ident ? 0.0 : (m1 ? q : -q);
    r = ident ? (m1 ? b : a) : rs * unsc;
}

__device__ __forceinline__ void givens(double a, double b, int mode, double &c, double &s, double &r)
{
    if (mode == 1)
        givens_m<1>(a, b, c, s, r);
    else
        givens_m<2>(a, b, c, s, r);
}

__device__ __forceinline__ void rot(double c, double s, double &x, double &y)
{
    double x0 = x, y0 = y;
    x = fma(c, x0, -(s * y0));
    y = fma(s, x0, c * y0);
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
        A = gptr(h->Q); x = gptr(h->bst) + (int64_t)pass * m; out = gptr(h->u); rows = m; ld = h->ldq;
    } else {
        tile -= qt;
        A = gptr(h->P); x = gptr(h->cst) + (int64_t)pass * n; out = gptr(h->v); rows = n; ld = h->ldp;
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

// ---- generation -------------------------------------------------------------------

// Band storage: band_row (device.h).  Entries outside the band read as zero
// and are never written: the schedule keeps them zero.

// Chain descriptor held in registers (GenChain fields).
struct ChainReg {
    int type, param, len, tau0;
    int64_t slot0, slot1;
};

__device__ __forceinline__ ChainReg load_chain(const GenChain *chains, int idx)
{
    const GLOBAL int *p = (const GLOBAL int *)gptr(chains) + 8 * idx;
    const GLOBAL int64_t *q = (const GLOBAL int64_t *)(p + 4);
    ChainReg c;
    c.type = p[0];
    c.param = p[1];
    c.len = p[2];
    c.tau0 = p[3];
    c.slot0 = q[0];
    c.slot1 = q[1];
    return c;
}

// A use that makes the compiler wait for a chain's loads at this point.  The
// vector memory counter also counts the coefficient stores, so a wait for a
// load left in flight across the tick loop would wait for the previous
// tick's store in every tick.
__device__ __forceinline__ void settle(const ChainReg &c)
{
    asm volatile("" ::"v"(c.type), "v"(c.param), "v"(c.len), "v"(c.tau0), "v"(c.slot0), "v"(c.slot1));
}

// Ticks between refills of a thread's prefetched chain descriptor.
constexpr int kRefill = 32;

__device__ __forceinline__ int band_cell(int r, int c)
{
    return band_row(r) + (c - r) + 2;
}

// Rotation s of chain g, decoded into band pointers.
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
// matching u or v pair.
//
// Consecutive rotations of a chain share two window pairs: in phase 1 pairs
// w_0, w_1 of one rotation are w_3, w_4 of the next, in phase 2 the reverse.
// The window is kept in the order (w_3, w_4, w_2, w_0, w_1) in phase 1 and
// (w_0, ..., w_4) in phase 2, so slots 0 and 1 are the pairs shared with the
// previous rotation and slots 3 and 4 those shared with the next, and the
// next rotation's slots 0, 1 hold (x_3, y_3), (x_4, y_4) of this one's, in
// both phases and both directions.  The pair a rotation is generated from
// is slot 1 in phase 1 and slot 0 in phase 2, except at a chain's first
// rotation: the u or v pair in phase 1, slot 1 in phase 2.
//
// Rotations s and s + 2 of a chain have the same pattern three rows and
// columns further on: every band pointer moves by kBandStep3 doubles, the u
// or v pointer by 3 and the coefficient slot by K.
template <typename BP>
struct RotAddr {
    BP x[5], y[5];      // window pairs, in slot order
    BP vb;              // u or v pair (vb[0], vb[1])
    GLOBAL double *cs;  // coefficient slot (c, s)
};

template <typename BP>
__device__ __forceinline__ RotAddr<BP> decode(BP S, const ChainReg &g, int s, int K, int UO, int VO,
                                              GLOBAL double *csL, GLOBAL double *csR)
{
    const bool ph1 = g.type <= CH_P1B;
    const bool first = ph1 ? (g.type == CH_P1A) : (g.type == CH_P2A);
    const int ss = s + (first ? 1 : 0);
    const int odd = ss & 1;
    const int i0 = ph1 ? (first ? g.param + 1 : g.param) : (first ? g.param - 3 : g.param - 1);
    const int ii = ph1 ? i0 - 3 * (ss >> 1) : i0 + 3 * (ss >> 1);
    const int side = ph1 ? odd : 1 - odd;
    const int i = ph1 ? (odd ? ii - 1 : ii) : (odd ? ii + 3 : ii + 2);
    RotAddr<BP> d;
    d.vb = S + (side == 0 ? UO : VO) + i + 3;
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
    constexpr int ord1[5] = {3, 4, 2, 0, 1};
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        d.x[k] = S + (ph1 ? wx[ord1[k]] : wx[k]);
        d.y[k] = S + (ph1 ? wy[ord1[k]] : wy[k]);
    }
    d.cs = (side == 0 ? csL + 2 * g.slot0 : csR + 2 * g.slot1) + (int64_t)(s >> 1) * 2 * K;
    return d;
}

template <typename BP>
__device__ __forceinline__ void advance(RotAddr<BP> &a, int db, int du, int64_t dcs)
{
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        a.x[q] += db;
        a.y[q] += db;
    }
    a.vb += du;
    a.cs += dcs;
}

// Generation of one pass for one handle per workgroup.  Thread l runs chains
// l, l + blockDim, ... (non-empty chains in schedule order); chain c performs
// its rotation s at tick tau0(c) + s, and a barrier separates ticks.  The host
// chose the start ticks so that two rotations touching a common band row, u or
// v entry are ordered as in the sequential schedule; in particular no other
// rotation touches a band entry between two consecutive rotations of a chain
// that share it, so the thread keeps the two shared pairs in registers
// (k0, k1) instead of writing and reading them back.  A tick reads three
// window pairs and the u or v pair, generates the rotation from registers and
// writes three pairs and the u or v pair; a chain's first tick also reads
// slots 0 and 1, its last also writes slots 3 and 4.
//
// Each thread keeps the pointers of its chain's next rotation at an even tick
// (ae) and at an odd tick (ao) and moves the set it has just used on to the
// chain's rotation two ticks later.
template <bool IN_LDS>
__global__ __launch_bounds__(kGenThreads) void gen_kernel(HandleDev *const *hs, Gate gate)
{
    extern __shared__ double smem[];
    if (gate.ranks && gate.pass >= gate.ranks[blockIdx.x]) return;
    const CONSTANT HandleDev *h = kptr(hs[blockIdx.x]);
    const int n = h->n, N = h->N;
    double *S = IN_LDS ? smem : h->band;
    // band pointers of the tick loop: LDS (32-bit) or global
    using BP = typename std::conditional<IN_LDS, LOCAL double *, GLOBAL double *>::type;
    const BP SB = (BP)S;
    const int UO = (int)band_doubles(N);  // u_i at S[UO + i + 3]
    const int VO = UO + (N + 8);          // v_j at S[VO + j + 3]
    const int tid = threadIdx.x;
    const int nt = blockDim.x;
    const int total = VO + (n + 8);
    for (int k = tid; k < total; k += nt) S[k] = 0.0;
    __syncthreads();
    for (int i = 1 + tid; i <= n; i += nt) {
        S[band_cell(i, i)] = h->d[i - 1];
        if (i < n) S[band_cell(i, i + 1)] = h->e[i - 1];
        S[VO + i + 3] = h->v[i - 1];
    }
    for (int i = 1 + tid; i <= N; i += nt) S[UO + i + 3] = h->u[i - 1];
    __syncthreads();

    const int K = h->K;
    const int nch = h->nchains;
    GLOBAL double *csL = gptr((double *)h->csL), *csR = gptr((double *)h->csR);
    const int64_t dcs = 2 * (int64_t)K;
    // Thread tid runs chains tid, tid + nt, ...; gn holds the next one when
    // `next` is set.  Descriptors are loaded and waited for before the loop,
    // every kRefill ticks, or (when a chain ends before a refill) at the
    // switch, so the tick body itself never waits on vector memory.
    int ci = tid;
    ChainReg g = {0, 0, 0, 0, 0, 0}, gn = {0, 0, 0, 0, 0, 0};
    bool next = false;
    if (ci < nch) g = load_chain(h->chains, ci);
    if (ci + nt < nch) {
        gn = load_chain(h->chains, ci + nt);
        next = true;
    }
    settle(g);
    settle(gn);

    RotAddr<BP> ae, ao;
    bool m1 = false, fold = false;
    int db = 0, du = 0;
    int tend = -1;
    auto start = [&]() {
        const RotAddr<BP> a0 = decode(SB, g, 0, K, UO, VO, csL, csR), a1 = decode(SB, g, 1, K, UO, VO, csL, csR);
        const bool odd0 = g.tau0 & 1;
        ae = odd0 ? a1 : a0;
        ao = odd0 ? a0 : a1;
        m1 = g.type <= CH_P1B;
        fold = g.type == CH_FOLD;
        db = m1 ? -kBandStep3 : kBandStep3;
        du = m1 ? -3 : 3;
        tend = g.tau0 + g.len - 1;
    };
    if (ci < nch) start();

    double kx0 = 0.0, kx1 = 0.0, ky0 = 0.0, ky1 = 0.0;  // slots 0, 1 carried from the previous rotation
    // One rotation with its window, for one phase (the phase is uniform
    // across a wavefront except where phase 2 starts, so a wavefront
    // normally runs one of the two bodies).
    auto rotate = [&](RotAddr<BP> &a, bool first, bool last, auto phase) {
        constexpr bool P1 = decltype(phase)::value;
        double xv[5], yv[5];
#pragma unroll
        for (int q = 2; q < 5; ++q) {
            xv[q] = *a.x[q];
            yv[q] = *a.y[q];
        }
        double ux = a.vb[0], uy = a.vb[1];
        // local copies: a select between captured variables would become a
        // load through a selected address
        xv[0] = kx0;
        xv[1] = kx1;
        yv[0] = ky0;
        yv[1] = ky1;
        double va = P1 ? xv[1] : xv[0], vb = P1 ? yv[1] : yv[0];
        if (first) {
            xv[0] = *a.x[0];
            xv[1] = *a.x[1];
            yv[0] = *a.y[0];
            yv[1] = *a.y[1];
            va = P1 ? ux : xv[1];
            vb = P1 ? uy : yv[1];
        }
        double c, sn, rr;
        givens_m<P1 ? 1 : 2>(va, vb, c, sn, rr);
#pragma unroll
        for (int q = 0; q < 5; ++q) rot(c, sn, xv[q], yv[q]);
        rot(c, sn, ux, uy);
        // the generating pair becomes (0, r) (mode 1) or (r, 0) (mode 2)
        if (P1) {
            ux = first ? 0.0 : ux;
            uy = first ? rr : uy;
            xv[1] = first ? xv[1] : 0.0;
            yv[1] = first ? yv[1] : rr;
        } else {
            xv[1] = first ? rr : xv[1];
            yv[1] = first ? 0.0 : yv[1];
            xv[0] = first ? xv[0] : rr;
            yv[0] = first ? yv[0] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            *a.x[q] = xv[q];
            *a.y[q] = yv[q];
        }
        a.vb[0] = ux;
        a.vb[1] = uy;
        if (last) {
            *a.x[3] = xv[3];
            *a.y[3] = yv[3];
            *a.x[4] = xv[4];
            *a.y[4] = yv[4];
        }
        kx0 = xv[3];
        kx1 = yv[3];
        ky0 = xv[4];
        ky1 = yv[4];
        // one 16-byte store of the rotation's (c, s)
        HIP_vector_base<double, 2>::Native_vec_ value;
        value[0] = c;
        value[1] = sn;
        *(GLOBAL HIP_vector_base<double, 2>::Native_vec_ *)a.cs = value;
    };

    auto tick = [&](RotAddr<BP> &a, int t) {
        const bool live = ci < nch && t >= g.tau0;
        if (live) {
            if (fold) {
                // u v^T now touches only (N-1, n) and (N, n)
                const int fa = band_cell(N - 1, n), fb = band_cell(N, n);
                S[fa] = fma(S[UO + N - 1 + 3], S[VO + n + 3], S[fa]);
                S[fb] = fma(S[UO + N + 3], S[VO + n + 3], S[fb]);
            } else if (m1) {
                rotate(a, t == g.tau0, t == tend, std::true_type{});
            } else {
                rotate(a, t == g.tau0, t == tend, std::false_type{});
            }
            if (t == tend) {
                ci += nt;
                if (next) {
                    g = gn;
                    next = false;
                } else if (ci < nch) {
                    g = load_chain(h->chains, ci);
                    settle(g);
                }
                if (ci < nch) start();
            } else {
                advance(a, db, du, dcs);
            }
        }
        if (((t + 1) & (kRefill - 1)) == 0 && !next && ci + nt < nch) {
            gn = load_chain(h->chains, ci + nt);
            settle(gn);
            next = true;
        }
        __syncthreads();
    };

    const int ticks = (int)h->ticks;
    int t = 0;
    for (; t + 1 < ticks; t += 2) {
        tick(ae, t);
        tick(ao, t + 1);
    }
    if (t < ticks) tick(ae, t);

    for (int i = 1 + tid; i <= n; i += nt) {
        h->d[i - 1] = S[band_cell(i, i)];
        if (i < n) h->e[i - 1] = S[band_cell(i, i + 1)];
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
    const int nb1 = h->nb1, nb2 = h->nb2;
    if (pid < qp) {
        const int row0 = pid * PH + lane;
        GLOBAL double *Q = gptr(h->Q);
        if (m > n && w == 0) {
#pragma unroll
            for (int r = 0; r < R; ++r) spike_apply(Q, h->ldq, m, n, row0 + 64 * r, kptr((const double *)h->csSp));
        }
        __syncthreads();
        for (int b = 0; b < nb1; ++b) {
            const BlockDesc bd = load_block(h->blkL, b);
            sweep<K0, NW, R, 0>(Q, h->ldq, m, row0, kptr((const double *)h->csL) + 2 * bd.off, bd, ring, w, lane);
            __syncthreads();
        }
        for (int b = nb1; b < nb1 + nb2; ++b) {
            const BlockDesc bd = load_block(h->blkL, b);
            sweep<K0, NW, R, 2>(Q, h->ldq, m, row0, kptr((const double *)h->csL) + 2 * bd.off, bd, ring, w, lane);
            __syncthreads();
        }
    } else {
        const int row0 = (pid - qp) * PH + lane;
        GLOBAL double *P = gptr(h->P);
        for (int b = 0; b < nb1; ++b) {
            const BlockDesc bd = load_block(h->blkR, b);
            sweep<K0, NW, R, 1>(P, h->ldp, n, row0, kptr((const double *)h->csR) + 2 * bd.off, bd, ring, w, lane);
            __syncthreads();
        }
        for (int b = nb1; b < nb1 + nb2; ++b) {
            const BlockDesc bd = load_block(h->blkR, b);
            sweep<K0, NW, R, 3>(P, h->ldp, n, row0, kptr((const double *)h->csR) + 2 * bd.off, bd, ring, w, lane);
            __syncthreads();
        }
    }
}

// ---- staged application ---------------------------------------------------------
//
// A workgroup of NW compute wavefronts and one memory wavefront (index NW).
// The compute wavefronts run the register-window sweep above with LDS
// traffic only: wavefront w takes its new columns from ring w and hands its
// finished columns to ring w + 1; the coefficients of each front come from a
// coefficient ring in LDS (one broadcast read per rotation).  The memory
// wavefront feeds ring 0 and the coefficient ring from global memory, DL
// fronts ahead, and writes the columns arriving in ring NW back to Q or P.
// Compute wavefronts therefore issue no global or scalar memory operation in
// their loop, and none of their waits depends on a global-memory latency.
template <int K0, int NW, int R>
struct Staged {
    static constexpr int U = K0 + 3, WSZ = 3 * U, S = U, K = K0 * NW;
    static constexpr int RC = ring_cols(K0);
    static constexpr int RING = RC * 64 * R;                  // doubles per ring
    static constexpr int COEF = (NW + 1) * RING;              // offset of the coefficient ring
    static constexpr int LDS_DOUBLES = COEF + 3 * K * 2;      // 3 fronts of K pairs
    static constexpr int DL = U / 3;                          // memory prefetch depth, U % DL == 0
    static constexpr int NCI = (K + 63) / 64;                 // coefficient loads per front
    static_assert(U % 3 == 0 && U % DL == 0 && (3 * U) % RC == 0, "static ring slots");
};

template <int K0, int NW, int R, int MODE>
__device__ __forceinline__ void sweep_compute(const BlockDesc bd, double *lds, int w, int lane)
{
    using T = Staged<K0, NW, R>;
    constexpr int U = T::U, WSZ = T::WSZ, S = T::S, K = T::K, RC = T::RC;
    constexpr bool DESC = MODE < 2;
    const int lmax = bd.lmax;
    if (lmax < 0) return;
    const int nfront = bd.nfront;
    const int lam_hi = lmax + 1;
    double buf[R][WSZ];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int i = 0; i < WSZ; ++i) buf[r][i] = 0.0;
    const double *rin = lds + w * T::RING + lane;
    double *rout = lds + (w + 1) * T::RING + lane;
    const double2 *coef = (const double2 *)(lds + T::COEF) + w * K0;
    constexpr FrontOrder ord = front_order(MODE, K, K0);
    const int flush_end = lam_hi / 3 + K0 - 1;
    const int nchunk = nfront / U;
    int live_end = w + (flush_end + U) / U;
    live_end = live_end < nchunk ? live_end : nchunk;
    auto idle = [&](int chunks) {
        for (int c = 0; c < chunks * U; ++c) __syncthreads();
    };
    __syncthreads();  // the memory wavefront's prologue is in LDS
    idle(w);
    for (int F0 = w * S; F0 < live_end * U; F0 += U) {
#pragma unroll
        for (int phi = 0; phi < U; ++phi) {
            const int F = F0 + phi;
            const int f = F - w * S;
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
            // front F's coefficients sit in slot F mod 3 (F0 is a multiple of 3)
            const double2 *cf = coef + (phi % 3) * K;
#pragma unroll
            for (int p = 0; p < K0; ++p) {
                const int t = ord.t[p];
                const int l0 = 3 * (phi - t) + rho_of(MODE, K, t);
                const int sx = pmod(l0 + (DESC ? 1 : 0), WSZ);
                const int sy = pmod(l0 + (DESC ? 0 : 1), WSZ);
                const double2 cv = cf[p];
#pragma unroll
                for (int r = 0; r < R; ++r) rot(cv.x, cv.y, buf[r][sx], buf[r][sy]);
            }
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int r = 0; r < R; ++r)
                    rout[(pmod(3 * (phi - K0 + 1) + k, RC) * R + r) * 64] = buf[r][pmod(3 * (phi - K0 + 1) + k, WSZ)];
            __syncthreads();
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int j = -3 * (K0 - 1); j <= 3; ++j) asm volatile("" : "+v"(buf[r][pmod(3 * phi + j, WSZ)]));
        }
    }
    idle(nchunk - (live_end > w ? live_end : w));
}

template <int K0, int NW, int R, int MODE>
__device__ __forceinline__ void sweep_memory(GLOBAL double *__restrict__ X, int ld, int ncols, int row0,
                                             const CONSTANT double *cs, const BlockDesc bd, double *lds, int lane)
{
    using T = Staged<K0, NW, R>;
    constexpr int U = T::U, S = T::S, K = T::K, RC = T::RC, DL = T::DL, NCI = T::NCI;
    constexpr bool DESC = MODE < 2;
    constexpr int DIR = DESC ? -1 : 1;
    const int lmax = bd.lmax;
    if (lmax < 0) return;
    const int nfront = bd.nfront;
    const int base = bd.base;
    const int lam_hi = lmax + 1;
    const int lam_lo = DESC ? (base - ncols > 0 ? base - ncols : 0) : 0;
    const int col0 = base - 1;
    double *rw = lds + lane;                               // ring 0
    const double *rr = lds + NW * T::RING + lane;          // ring NW
    double *coef = lds + T::COEF;  // pairs (c, s)
    const GLOBAL double *cg = (const GLOBAL double *)(uintptr_t)cs;
    auto colptr = [&](int lam) -> const GLOBAL double * {
        int c = col0 + DIR * lam;
        c = c < 0 ? 0 : (c >= ncols ? ncols - 1 : c);
        return X + (int64_t)c * ld;
    };
    // FIFO entry for front Fl (written to LDS during front Fl): the columns
    // 3 Fl + 7 .. 3 Fl + 9 that wavefront 0 reads at front Fl + 1 (for its
    // front Fl + 2), and the coefficients of front Fl + 1.
    double colf[DL][3][R];
    double cof[DL][NCI][2];
    auto load_entry = [&](int slot, int Fl) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const GLOBAL double *cp = colptr(3 * Fl + 7 + k);
#pragma unroll
            for (int r = 0; r < R; ++r) colf[slot][k][r] = cp[row0 + 64 * r];
        }
        int Fc = Fl + 1 < nfront ? Fl + 1 : nfront - 1;
        const GLOBAL double *cp = cg + 2 * (int64_t)Fc * K;
#pragma unroll
        for (int i = 0; i < NCI; ++i) {
            const int q = lane + 64 * i < K ? lane + 64 * i : K - 1;
            cof[slot][i][0] = cp[2 * q];
            cof[slot][i][1] = cp[2 * q + 1];
        }
    };
    // prologue: columns 0..6 and front 0's coefficients, then the FIFO
    {
#pragma unroll
        for (int k = 0; k <= 6; ++k) {
            const GLOBAL double *cp = colptr(k);
#pragma unroll
            for (int r = 0; r < R; ++r) rw[(k * R + r) * 64] = cp[row0 + 64 * r];
        }
#pragma unroll
        for (int i = 0; i < NCI; ++i)
            if (lane + 64 * i < K) {
                coef[2 * (lane + 64 * i)] = cg[2 * (lane + 64 * i)];
                coef[2 * (lane + 64 * i) + 1] = cg[2 * (lane + 64 * i) + 1];
            }
    }
#pragma unroll
    for (int j = 0; j < DL; ++j) load_entry(j, j);
    __syncthreads();
    for (int F0 = 0; F0 < nfront; F0 += U) {
#pragma unroll
        for (int phi = 0; phi < U; ++phi) {
            const int F = F0 + phi;
            const int slot = phi % DL;
            // columns wavefront 0 reads at front F + 1, coefficients of front F + 1
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int r = 0; r < R; ++r) rw[(pmod(3 * phi + 7 + k, RC) * R + r) * 64] = colf[slot][k][r];
#pragma unroll
            for (int i = 0; i < NCI; ++i)
                if (lane + 64 * i < K) {
                    double *d = coef + 2 * (((phi + 1) % 3) * K + lane + 64 * i);
                    d[0] = cof[slot][i][0];
                    d[1] = cof[slot][i][1];
                }
            load_entry(slot, F + DL);
            // columns the last compute wavefront finished at front F - 1
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int lam = 3 * (F - 1 - (NW - 1) * S - K0 + 1) + k;
                if (lam >= lam_lo && lam <= lam_hi) {
                    GLOBAL double *cp = X + (int64_t)(col0 + DIR * lam) * ld;
#pragma unroll
                    for (int r = 0; r < R; ++r) cp[row0 + 64 * r] = rr[(pmod(3 * phi - 3 * K0 + k, RC) * R + r) * 64];
                }
            }
            __syncthreads();
        }
    }
}

template <int K0, int NW, int R>
__global__ __launch_bounds__(64 * (NW + 1)) __attribute__((amdgpu_waves_per_eu(R == 2 ? 2 : (K0 > 12 ? 3 : 4))))
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
    const int nb1 = h->nb1, nb2 = h->nb2;
    const bool onQ = pid < qp;
    const int row0 = (onQ ? pid : pid - qp) * PH + lane;
    GLOBAL double *X = gptr(onQ ? h->Q : h->P);
    const int ld = onQ ? h->ldq : h->ldp;
    const int ncols = onQ ? m : n;
    const BlockDesc *blk = onQ ? h->blkL : h->blkR;
    const CONSTANT double *cs = kptr((const double *)(onQ ? h->csL : h->csR));
    if (onQ && m > n && w == 0) {
#pragma unroll
        for (int r = 0; r < R; ++r) spike_apply(X, ld, m, n, row0 + 64 * r, kptr((const double *)h->csSp));
    }
    __syncthreads();
    for (int b = 0; b < nb1 + nb2; ++b) {
        const BlockDesc bd = load_block(blk, b);
        const CONSTANT double *cb = cs + 2 * bd.off;
        if (w == NW) {
            if (b < nb1) {
                if (onQ) sweep_memory<K0, NW, R, 0>(X, ld, ncols, row0, cb, bd, lds, lane);
                else sweep_memory<K0, NW, R, 1>(X, ld, ncols, row0, cb, bd, lds, lane);
            } else {
                if (onQ) sweep_memory<K0, NW, R, 2>(X, ld, ncols, row0, cb, bd, lds, lane);
                else sweep_memory<K0, NW, R, 3>(X, ld, ncols, row0, cb, bd, lds, lane);
            }
        } else {
            if (b < nb1) {
                if (onQ) sweep_compute<K0, NW, R, 0>(bd, lds, w, lane);
                else sweep_compute<K0, NW, R, 1>(bd, lds, w, lane);
            } else {
                if (onQ) sweep_compute<K0, NW, R, 2>(bd, lds, w, lane);
                else sweep_compute<K0, NW, R, 3>(bd, lds, w, lane);
            }
        }
        __syncthreads();
    }
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

hipError_t prepare_kernels()
{
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)gen_kernel<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)kMaxGenLds);
        if (e != hipSuccess) return e;
        attr = true;
    }
    return hipSuccess;
}

hipError_t launch_gen(HandleDev *const *hs, int count, int64_t lds_bytes, bool in_lds, Gate gate, hipStream_t st)
{
    if (in_lds) {
        hipError_t e = prepare_kernels();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(gen_kernel<true>, dim3(count), dim3(kGenThreads), (size_t)lds_bytes, st, hs, gate);
    } else {
        hipLaunchKernelGGL(gen_kernel<false>, dim3(count), dim3(kGenThreads), 0, st, hs, gate);
    }
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
