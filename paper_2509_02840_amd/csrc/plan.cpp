// plan.cpp -- builds the schedule tables of one shape on the host.
//
// 1. The chains of a pass, in the order of Section 3.4 / Algorithm 2 (see
//    schedule.h), with their lengths.
// 2. Generation ticks.  Chains run concurrently, one per thread, one
//    rotation per tick.  A chain may start at tick tau0 only if every
//    rotation it performs comes strictly after every earlier rotation whose
//    band rows overlap (so every band entry sees its updates in schedule
//    order), and only once its thread has finished the previous chain.  The
//    earliest such tau0 is taken chain by chain.
// 3. Applier blocks for the left (Q) and right (P) rotation streams.
#include "plan.h"

#include <algorithm>
#include <climits>

namespace bdu {

static void add_chain(std::vector<GenChain> &v, int type, int param, int len)
{
    if (len <= 0) return;
    GenChain c;
    c.type = type;
    c.param = param;
    c.len = len;
    c.tau0 = 0;
    v.push_back(c);
}

// Start chunks of the staged applier's blocks on one side (ncols columns of
// Q or P).  The applier runs a launch's blocks back to back: compute
// wavefront w is live in block b during chunks [start_b + w, start_b + w +
// C_b) (chunks of U = K0 + 3 fronts, C_b = (lam_hi / 3 + K0 - 1 + U) / U,
// lam_hi = lmax + 1), so block b + 1 may start once every wavefront has
// finished block b (start_{b+1} >= start_b + C_b) -- and once the memory
// wavefront, which moves every column between device memory and the
// pipeline, keeps each column's order across blocks: it loads local column
// lam of block b at front start_b U + max(-1, (lam - 7) / 3 - DL) (-1: the
// block's prologue, the front before it starts; columns 0..6 too) and stores it at
// front start_b U + lam / 3 + (NW - 1) U + K0.  A load of a column comes at
// least DL + 3 fronts after every earlier block's store of it (by then the
// store has completed: vector memory operations complete in issue order and
// the memory wavefront has waited for a load issued after it), and a store
// after every earlier load and store of it.  Each block takes the earliest
// start that satisfies these against all earlier blocks of the side.
static void stage_starts(std::vector<BlockDesc> &blk, int64_t ncols, int K0, int NW)
{
    const int U = K0 + 3, DL = U / 3, margin = DL + 3;
    const int64_t none = INT64_MIN / 4;
    std::vector<int64_t> st((size_t)ncols, none), ldf((size_t)ncols, none);
    int64_t s = 0;  // earliest start of the next block (chunks)
    for (BlockDesc &d : blk) {
        d.pad = 0;
        if (d.lmax < 0) {
            d.start = (int32_t)s;
            continue;
        }
        const int dir = d.phase == 1 ? -1 : 1, col0 = d.base - 1, lam_hi = d.lmax + 1;
        const int C = (lam_hi / 3 + K0 - 1 + U) / U;
        auto load_off = [&](int lam) { return lam < 7 ? -1 : std::max(-1, (lam - 7) / 3 - DL); };
        auto store_off = [&](int lam) { return lam / 3 + (NW - 1) * U + K0; };
        int64_t need = s * U;  // earliest first front
        for (int lam = 0; lam <= lam_hi; ++lam) {
            const int64_t c = col0 + (int64_t)dir * lam;
            if (c < 0 || c >= ncols) continue;
            if (st[c] != none) need = std::max<int64_t>(need, st[c] + margin - load_off(lam));
            need = std::max<int64_t>(need, std::max(ldf[c], st[c]) + 1 - store_off(lam));
        }
        const int64_t start = (need + U - 1) / U;
        d.start = (int32_t)start;
        for (int lam = 0; lam <= lam_hi; ++lam) {
            const int64_t c = col0 + (int64_t)dir * lam;
            if (c < 0 || c >= ncols) continue;
            ldf[c] = std::max<int64_t>(ldf[c], start * U + load_off(lam));
            st[c] = start * U + store_off(lam);
        }
        s = start + C;
    }
}

// Segments of a single-handle pass (more segments hide more of the
// application behind generation; each costs a generation launch with its
// band save and reload and an applier launch).  Measured on one stream:
// 8 are best from n = 257 up, 4 below (n = 129: 0.82 ms against 0.85).
constexpr int kSegments = 8, kSegmentsSmall = 4;

std::unique_ptr<Plan> build_plan(int64_t m, int64_t n, int K0, int NW, int gen_threads)
{
    auto P = std::make_unique<Plan>();
    P->m = m;
    P->n = n;
    P->N = (m == n) ? n : n + 1;
    P->K0 = K0;
    P->NW = NW;
    P->K = K0 * NW;
    P->S = K0 + 3;
    P->L = gen_threads;
    const int N = (int)P->N, nn = (int)n;

    // ---- chains ---------------------------------------------------------
    std::vector<GenChain> &ch = P->chains;
    for (int k = 1; k <= nn - 1; ++k) {
        add_chain(ch, CH_P1A, k, 1 + len_up(k - 2));
        if (k <= N - 2) add_chain(ch, CH_P1B, k, 1 + (k >= 2 ? 1 + len_up(k - 3) : 0));
    }
    add_chain(ch, CH_FOLD, 0, 1);
    for (int j = 1; j <= nn; ++j) {
        if (j + 1 <= N) add_chain(ch, CH_P2A, j, 1 + len_down(j, nn, N));
        if (j + 2 <= nn) add_chain(ch, CH_P2B, j, 1 + (j + 3 <= N ? 1 + len_down(j + 2, nn, N) : 0));
    }
    P->nspike = (m > n) ? (m - n - 1) : 0;

    // ---- generation ticks -------------------------------------------------
    // A chain starts at the earliest tick at which each of its rotations runs
    // after every earlier rotation (schedule order) that touches one of the
    // same entries: a band cell (rows x columns within offsets -2..3), u or v.
    // A left rotation on rows (i, i+1) touches columns i-1..i+3 of them and
    // u_i, u_{i+1}; a right rotation on columns (j, j+1) rows j-2..j+2 and
    // v_j, v_{j+1} (the only entries the schedule can make nonzero there).
    const int off = 5;  // rows and columns -4 .. N+5
    const int W = N + 12;
    std::vector<int64_t> lastcell((size_t)W * 6, -1), lastu(W, -1), lastv(W, -1);
    auto cells = [&](const Rot &r, auto &&fn) {
        if (r.side == 0) {
            for (int row = r.i; row <= r.i + 1; ++row)
                for (int c = r.i - 1; c <= r.i + 3; ++c)
                    if (c - row >= -2 && c - row <= 3) fn(lastcell[(size_t)(row + off) * 6 + (c - row + 2)]);
            fn(lastu[r.i + off]);
            fn(lastu[r.i + 1 + off]);
        } else {
            for (int row = r.i - 2; row <= r.i + 2; ++row)
                for (int c = r.i; c <= r.i + 1; ++c)
                    if (c - row >= -2 && c - row <= 3) fn(lastcell[(size_t)(row + off) * 6 + (c - row + 2)]);
            fn(lastv[r.i + off]);
            fn(lastv[r.i + 1 + off]);
        }
    };
    auto fold_cells = [&](auto &&fn) {  // (N-1, n), (N, n), u_{N-1}, u_N, v_n
        fn(lastcell[(size_t)(N - 1 + off) * 6 + (nn - (N - 1) + 2)]);
        fn(lastcell[(size_t)(N + off) * 6 + (nn - N + 2)]);
        fn(lastu[N - 1 + off]);
        fn(lastu[N + off]);
        fn(lastv[nn + off]);
    };
    // With fewer chains than threads every chain gets its own thread, so
    // the workgroup only needs that many (rounded to whole wavefronts):
    // fewer wavefronts meet at every tick's barrier.
    const int L = (int)std::min<int64_t>(gen_threads, std::max<int64_t>(64, ((int64_t)ch.size() + 63) / 64 * 64));
    P->L = L;
    std::vector<int64_t> lane_free(L, 0);
    int64_t tend = 0;
    for (size_t c = 0; c < ch.size(); ++c) {
        GenChain &g = ch[c];
        int64_t tau0 = 0;
        for (int s = 0; s < g.len; ++s) {
            auto need = [&](int64_t &t) { tau0 = std::max(tau0, t + 1 - s); };
            if (g.type == CH_FOLD) fold_cells(need);
            else cells(decode(g.type, g.param, s), need);
        }
        int lane = (int)(c % L);
        tau0 = std::max(tau0, lane_free[lane]);
        for (int s = 0; s < g.len; ++s) {
            auto mark = [&](int64_t &t) { t = std::max(t, tau0 + s); };
            if (g.type == CH_FOLD) {
                fold_cells(mark);
            } else {
                Rot r = decode(g.type, g.param, s);
                cells(r, mark);
                if (r.side == 0) ++P->nleft; else ++P->nright;
            }
        }
        lane_free[lane] = tau0 + g.len;
        g.tau0 = (int32_t)tau0;
        tend = std::max(tend, tau0 + g.len);
    }
    P->ticks = tend;
    // Phase 1 (with the fold) ends at the tick its last chain finishes; the
    // pass can be generated in two parts split there when no chain is in
    // flight at that tick and no phase-2 chain starts before it (then the
    // second part needs only the band, and phase 1 can be applied while
    // phase 2 is generated).
    int64_t p1end = 0;
    for (const GenChain &g : ch)
        if (g.type <= CH_P1B || g.type == CH_FOLD) p1end = std::max<int64_t>(p1end, g.tau0 + g.len);
    bool clean = p1end > 0 && p1end < tend;
    for (const GenChain &g : ch) {
        if (g.tau0 < p1end && g.tau0 + g.len > p1end) clean = false;
        if (g.type >= CH_P2A && g.tau0 < p1end) clean = false;
    }
    P->split = clean ? p1end : 0;

    // ---- applier blocks -------------------------------------------------
    const int K = P->K, S = P->S;
    P->nb1 = (2 * (nn - 1) + K - 1) / K;
    P->nb2 = (2 * nn + K - 1) / K;
    for (int side = 0; side < 2; ++side) {
        int64_t pos = 0;
        for (int ph = 1; ph <= 2; ++ph) {
            int nb = ph == 1 ? P->nb1 : P->nb2;
            for (int b = 0; b < nb; ++b) {
                BlockDesc d;
                d.phase = ph;
                d.base = block_base(ph, b, K);
                if (ph == 1) {
                    d.lmax = d.base - 2;  // lowest pair is 1
                } else {
                    int hi = side == 0 ? N - 1 : nn - 1;
                    d.lmax = hi - d.base;
                }
                if (d.lmax < 0) {
                    d.lmax = -1;
                    d.nfront = 0;
                } else {
                    // every wavefront sweeps until its last column has left
                    const int fend = d.lmax / 3 + K0 + 1;
                    const int Fend = fend + (NW - 1) * S;
                    d.nfront = ((Fend + 1 + S - 1) / S) * S;
                }
                d.off = pos;
                pos += (int64_t)d.nfront * K;
                P->blocks[side].push_back(d);
            }
        }
        P->slots[side] = pos;
        stage_starts(P->blocks[side], side == 0 ? m : n, K0, NW);
    }
    // first slot of each chain on each side (same formula the applier reads)
    for (GenChain &g : ch) {
        g.slot[0] = g.slot[1] = -1;
        if (g.type == CH_FOLD) continue;
        const int ph = chain_phase(g.type), tg = chain_in_phase(g.type, g.param);
        const int b = tg / K, tin = tg % K, w = tin / K0, tl = tin % K0;
        for (int s = 0; s < g.len && s < 2; ++s) {
            const Rot r = decode(g.type, g.param, s);
            const BlockDesc &bd = P->blocks[r.side][(ph == 1 ? 0 : P->nb1) + b];
            const int lam0 = lam0_of_pair(ph, bd.base, r.i);
            const int pos = front_order(2 * (ph - 1) + r.side, K, K0).pos[tl];
            g.slot[r.side] = bd.off + (int64_t)(lam0 / 3 + tl + w * S) * K + w * K0 + pos;
        }
    }
    // the first two rotations of each chain, decoded for the in-LDS
    // generation kernel (in the order of its even- and odd-tick sets)
    {
        const int uo = (int)band_doubles(N), vo = uo + (N + 8);
        if ((int64_t)vo + nn + 8 <= 65536) {
            P->starts.resize(ch.size());
            for (size_t c = 0; c < ch.size(); ++c) {
                const GenChain &g = ch[c];
                GenStart &st = P->starts[c];
                for (uint32_t &o : st.off) o = 0;
                st.sides = 0;
                if (g.type == CH_FOLD) continue;
                const int se = (g.tau0 & 1) ? 1 : 0;
                for (int set = 0; set < 2; ++set) {
                    const int s = set == 0 ? se : 1 - se;
                    if (s >= g.len) continue;
                    const RotOff o = rot_offsets(g.type, g.param, s, uo, vo);
                    const int v[11] = {o.x[0], o.x[1], o.x[2], o.x[3], o.x[4], o.y[0], o.y[1], o.y[2], o.y[3], o.y[4],
                                       o.vb};
                    for (int k = 0; k < 11; ++k) st.off[k] |= (uint32_t)v[k] << (16 * set);
                    st.sides |= o.side << set;
                }
            }
        }
    }
    // ---- segments of a pass ---------------------------------------------
    // Applier block b (phase-1 blocks, then phase-2 blocks) holds the chains
    // of in-phase index [bK, bK + K) of its phase on both sides; blocks
    // [0, c) are complete at the tick their last chain ends.  Segment k ends
    // at such a tick for the block cut c_k (cuts spread evenly over the
    // blocks, the last at all of them), so its application can run while
    // the next segment is generated.  Chains may be in flight at a segment
    // end: the generator saves their carried pairs.
    {
        const int nbt = P->nb1 + P->nb2;
        std::vector<int64_t> done(nbt, 0);
        for (const GenChain &g : ch) {
            if (g.type == CH_FOLD) continue;
            const int b = chain_in_phase(g.type, g.param) / K + (chain_phase(g.type) == 1 ? 0 : P->nb1);
            done[b] = std::max<int64_t>(done[b], g.tau0 + g.len);
        }
        for (int b = 1; b < nbt; ++b) done[b] = std::max(done[b], done[b - 1]);
        const int want = std::min(nn >= 256 ? kSegments : kSegmentsSmall, nbt);
        int64_t prev_t = 0;
        int prev_c = 0;
        for (int k = 1; k <= want; ++k) {
            const int c = k == want ? nbt : (int)((int64_t)nbt * k / want);
            const int64_t t = k == want ? P->ticks : done[c - 1];
            if (c <= prev_c || t <= prev_t || (k < want && t >= P->ticks)) continue;
            P->bcut[P->nseg] = c;
            P->tcut[P->nseg] = (int32_t)t;
            ++P->nseg;
            prev_c = c;
            prev_t = t;
        }
        if (P->nseg == 0 || P->bcut[P->nseg - 1] != nbt || P->tcut[P->nseg - 1] != P->ticks) P->nseg = 0;
        for (const GenChain &g : ch)
            if (g.type == CH_FOLD)
                while (P->fold_seg + 1 < P->nseg && g.tau0 >= P->tcut[P->fold_seg]) ++P->fold_seg;
    }
    return P;
}

}  // namespace bdu
