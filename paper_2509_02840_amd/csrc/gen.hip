// gen.hip -- gfx950 kernel generating the rotations of one pass of the
// Givens bidiagonal update (Brust & Saunders, Section 3.4, Algorithm 2):
// phases 1 and 2 on the band of the working matrix, held in LDS (or global
// memory for large n), one thread per chain in flight, one rotation per
// tick, ticks separated by barriers.  FP64 throughout.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device.h"
#include "kernels.h"
#include "primitives.h"
#include "schedule.h"

namespace bdu {

// ---- generation -------------------------------------------------------------------

// Band storage: band_row (device.h).  Entries outside the band read as zero
// and are never written: the schedule keeps them zero.

// Chain descriptor held in registers (GenChain fields, and for the in-LDS
// kernel the chain's GenStart record).
struct ChainReg {
    int type, param, len, tau0;
    int64_t slot0, slot1;
    uint32_t so[11];
    int sides;
};

template <bool IN_LDS>
__device__ __forceinline__ ChainReg load_chain(const GenChain *chains, const GenStart *starts, int idx)
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
    if constexpr (IN_LDS) {
        const GLOBAL uint32_t *r = (const GLOBAL uint32_t *)gptr(starts) + 12 * idx;
#pragma unroll
        for (int k = 0; k < 11; ++k) c.so[k] = r[k];
        c.sides = (int)r[11];
    } else {
#pragma unroll
        for (int k = 0; k < 11; ++k) c.so[k] = 0;
        c.sides = 0;
    }
    return c;
}

// A use that makes the compiler wait for a chain's loads at this point.  The
// vector memory counter also counts the coefficient stores, so a wait for a
// load left in flight across the tick loop would wait for the previous
// tick's store in every tick.
template <bool IN_LDS>
__device__ __forceinline__ void settle(const ChainReg &c)
{
    asm volatile("" ::"v"(c.type), "v"(c.param), "v"(c.len), "v"(c.tau0), "v"(c.slot0), "v"(c.slot1));
    if constexpr (IN_LDS) {
#pragma unroll
        for (int k = 0; k < 11; ++k) asm volatile("" ::"v"(c.so[k]));
        asm volatile("" ::"v"(c.sides));
    }
}

// Ticks between refills of a thread's prefetched chain descriptor.
constexpr int kRefill = 32;

__device__ __forceinline__ int band_cell(int r, int c)
{
    return band_row(r) + (c - r) + 2;
}

// Rotation s of chain g as band pointers (the offsets of rot_offsets):
// the pair a rotation is generated from is slot 1 in phase 1 and slot 0 in
// phase 2, except at a chain's first rotation: the u or v pair in phase 1,
// slot 1 in phase 2.  The next rotation's slots 0, 1 hold (x_3, y_3),
// (x_4, y_4) of this one's, in both phases and both directions.
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
    const RotOff o = rot_offsets(g.type, g.param, s, UO, VO);
    RotAddr<BP> d;
    d.vb = S + o.vb;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        d.x[k] = S + o.x[k];
        d.y[k] = S + o.y[k];
    }
    d.cs = (o.side == 0 ? csL + 2 * g.slot0 : csR + 2 * g.slot1) + (int64_t)(s >> 1) * 2 * K;
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
    // a batch runs as many segments as its largest plan has; this
    // handle's pass may have ended already
    if (gate.part >= 3 && gate.part - 3 >= h->nseg) return;
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
    // A part after the first continues from the band the previous one left
    // (in device memory, or the image of the LDS band saved there);
    // otherwise start from d, e, u and v.  Parts: 0 all ticks, 1 phase 1,
    // 2 phase 2, 3 + k segment k.
    const int part = gate.part;
    const int ticks = (int)h->ticks, split = (int)h->split;
    int t_begin = 0, t_end = ticks;
    if (part == 1) t_end = split;
    if (part == 2) t_begin = split;
    if (part >= 3) {
        const int k = part - 3;
        t_begin = k == 0 ? 0 : h->tcut[k - 1];
        t_end = h->tcut[k];
    }
    if (t_begin > 0) {
        if (IN_LDS)
            for (int k = tid; k < total; k += nt) S[k] = h->band[k];
        // u_N, the spike's survivor, is read only by the fold: a pass may
        // start generating before the spike has finished (the first segment
        // then read u_N early) and let only the fold's segment wait for it,
        // so every later segment takes u_N afresh
        if (N > n && tid == 0) S[UO + N + 3] = h->u[N - 1];
        __syncthreads();
    } else {
        for (int k = tid; k < total; k += nt) S[k] = 0.0;
        __syncthreads();
        for (int i = 1 + tid; i <= n; i += nt) {
            S[band_cell(i, i)] = h->d[i - 1];
            if (i < n) S[band_cell(i, i + 1)] = h->e[i - 1];
            S[VO + i + 3] = h->v[i - 1];
        }
        for (int i = 1 + tid; i <= N; i += nt) S[UO + i + 3] = h->u[i - 1];
        __syncthreads();
    }

    const int K = h->K;
    const int nch = h->nchains;
    GLOBAL double *csL = gptr((double *)h->csL), *csR = gptr((double *)h->csR);
    const int64_t dcs = 2 * (int64_t)K;
    // Thread tid runs chains tid, tid + nt, ...; gn holds the next one when
    // `next` is set.  Descriptors are loaded and waited for before the loop,
    // every kRefill ticks, or (when a chain ends before a refill) at the
    // switch, so the tick body itself never waits on vector memory.
    int ci = tid;
    ChainReg g = {}, gn = {};
    bool next = false;
    if (ci < nch) g = load_chain<IN_LDS>(h->chains, h->starts, ci);
    settle<IN_LDS>(g);
    // part 2: skip the chains that finished before it (none is in flight at
    // the split)
    while (ci < nch && g.tau0 + g.len <= t_begin) {
        ci += nt;
        if (ci < nch) {
            g = load_chain<IN_LDS>(h->chains, h->starts, ci);
            settle<IN_LDS>(g);
        }
    }
    if (ci + nt < nch) {
        gn = load_chain<IN_LDS>(h->chains, h->starts, ci + nt);
        next = true;
    }
    settle<IN_LDS>(gn);

    RotAddr<BP> ae, ao;
    bool m1 = false, fold = false;
    int db = 0, du = 0;
    int tend = -1;
    auto start = [&]() {
        if constexpr (IN_LDS) {
            // both address sets as the host decoded them, already in even-
            // and odd-tick order
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                ae.x[k] = SB + (g.so[k] & 0xffffu);
                ao.x[k] = SB + (g.so[k] >> 16);
                ae.y[k] = SB + (g.so[5 + k] & 0xffffu);
                ao.y[k] = SB + (g.so[5 + k] >> 16);
            }
            ae.vb = SB + (g.so[10] & 0xffffu);
            ao.vb = SB + (g.so[10] >> 16);
            GLOBAL double *cl = csL + 2 * g.slot0, *cr = csR + 2 * g.slot1;
            ae.cs = (g.sides & 1) ? cr : cl;
            ao.cs = (g.sides & 2) ? cr : cl;
        } else {
            const RotAddr<BP> a0 = decode(SB, g, 0, K, UO, VO, csL, csR),
                              a1 = decode(SB, g, 1, K, UO, VO, csL, csR);
            const bool odd0 = g.tau0 & 1;
            ae = odd0 ? a1 : a0;
            ao = odd0 ? a0 : a1;
        }
        m1 = g.type <= CH_P1B;
        fold = g.type == CH_FOLD;
        db = m1 ? -kBandStep3 : kBandStep3;
        du = m1 ? -3 : 3;
        tend = g.tau0 + g.len - 1;
    };
    double kx0 = 0.0, kx1 = 0.0, ky0 = 0.0, ky1 = 0.0;  // slots 0, 1 carried from the previous rotation
    if (ci < nch) {
        start();
        if (g.tau0 < t_begin) {
            // in flight since an earlier segment: resume at rotation q with
            // the carried pairs that segment saved
            const int q = t_begin - g.tau0;
            const RotAddr<BP> aq = decode(SB, g, q, K, UO, VO, csL, csR),
                              aq1 = decode(SB, g, q + 1, K, UO, VO, csL, csR);
            const bool oddq = t_begin & 1;
            ae = oddq ? aq1 : aq;
            ao = oddq ? aq : aq1;
            kx0 = h->carry[4 * tid];
            kx1 = h->carry[4 * tid + 1];
            ky0 = h->carry[4 * tid + 2];
            ky1 = h->carry[4 * tid + 3];
        }
    }
    // wait for the carries here: a load still in flight at the tick loop
    // would make the loop wait on the vector memory counter in every tick,
    // and that counter also counts the coefficient stores
    asm volatile("" ::"v"(kx0), "v"(kx1), "v"(ky0), "v"(ky1));
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
        givens_fast<P1 ? 1 : 2>(va, vb, c, sn, rr);
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
                    g = load_chain<IN_LDS>(h->chains, h->starts, ci);
                    settle<IN_LDS>(g);
                }
                if (ci < nch) start();
            } else {
                advance(a, db, du, dcs);
            }
        }
        if (((t + 1) & (kRefill - 1)) == 0 && !next && ci + nt < nch) {
            gn = load_chain<IN_LDS>(h->chains, h->starts, ci + nt);
            settle<IN_LDS>(gn);
            next = true;
        }
        __syncthreads();
    };

    int t = t_begin;
    if (t < t_end && (t & 1)) {
        tick(ao, t);
        ++t;
    }
    for (; t + 1 < t_end; t += 2) {
        tick(ae, t);
        tick(ao, t + 1);
    }
    if (t < t_end) tick(ae, t);

    if (t_end < ticks) {
        // a later part continues: keep the band and the carries of a chain
        // still in flight (none at the end of phase 1)
        if (IN_LDS)
            for (int k = tid; k < total; k += nt) h->band[k] = S[k];
        if (ci < nch && g.tau0 < t_end) {
            h->carry[4 * tid] = kx0;
            h->carry[4 * tid + 1] = kx1;
            h->carry[4 * tid + 2] = ky0;
            h->carry[4 * tid + 3] = ky1;
        }
        return;
    }
    for (int i = 1 + tid; i <= n; i += nt) {
        h->d[i - 1] = S[band_cell(i, i)];
        if (i < n) h->e[i - 1] = S[band_cell(i, i + 1)];
    }
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

hipError_t launch_gen(HandleDev *const *hs, int count, int64_t lds_bytes, bool in_lds, int threads, Gate gate,
                      hipStream_t st)
{
    if (threads < 64 || threads > kGenThreads || threads % 64) return hipErrorInvalidValue;
    if (in_lds) {
        hipError_t e = prepare_kernels();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(gen_kernel<true>, dim3(count), dim3(threads), (size_t)lds_bytes, st, hs, gate);
    } else {
        hipLaunchKernelGGL(gen_kernel<false>, dim3(count), dim3(threads), 0, st, hs, gate);
    }
    return hipGetLastError();
}

}  // namespace bdu
