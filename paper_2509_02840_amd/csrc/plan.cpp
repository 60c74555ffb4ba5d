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
    const int off = 5;  // band-row line covers rows -4 .. N+5
    std::vector<int64_t> last(N + 12, -1);
    std::vector<int64_t> lane_free(gen_threads, 0);
    int64_t tend = 0;
    for (size_t c = 0; c < ch.size(); ++c) {
        GenChain &g = ch[c];
        int64_t tau0 = 0;
        for (int s = 0; s < g.len; ++s) {
            int lo, hi;
            if (g.type == CH_FOLD) {
                lo = N - 1;
                hi = N;
            } else {
                footprint(decode(g.type, g.param, s), &lo, &hi);
            }
            for (int x = lo; x <= hi; ++x) tau0 = std::max(tau0, last[x + off] + 1 - s);
        }
        int lane = (int)(c % gen_threads);
        tau0 = std::max(tau0, lane_free[lane]);
        for (int s = 0; s < g.len; ++s) {
            int lo, hi;
            if (g.type == CH_FOLD) {
                lo = N - 1;
                hi = N;
            } else {
                Rot r = decode(g.type, g.param, s);
                footprint(r, &lo, &hi);
                if (r.side == 0) ++P->nleft; else ++P->nright;
            }
            for (int x = lo; x <= hi; ++x) last[x + off] = std::max(last[x + off], tau0 + s);
        }
        lane_free[lane] = tau0 + g.len;
        g.tau0 = (int32_t)tau0;
        tend = std::max(tend, tau0 + g.len);
    }
    P->ticks = tend;

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
    return P;
}

}  // namespace bdu
