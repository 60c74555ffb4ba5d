// Builds the host schedule tables (plan.cpp) for many shapes and applier
// tilings under the sanitizers and checks their invariants: every rotation
// of every chain is counted once, chains start in order within their
// generation thread, every first slot lies inside its side's stream, blocks
// tile the streams in order, and the segment cuts rise to the last block and
// tick.  Exit status 0 when every check holds.
#include <stdio.h>

#include <algorithm>
#include <vector>

#include "../../paper_2509_02840_amd/csrc/plan.h"

static int g_fail = 0;
#define CHECK(c)                                                                          \
    do {                                                                                  \
        if (!(c)) {                                                                       \
            fprintf(stderr, "check failed at line %d (m %ld n %ld K0 %d NW %d): %s\n",     \
                    __LINE__, (long)m, (long)n, k0, nw, #c);                              \
            ++g_fail;                                                                     \
        }                                                                                 \
    } while (0)

int main()
{
    using namespace bdu;
    const long shapes[][2] = {{2, 2}, {3, 2}, {3, 3}, {4, 2}, {5, 5}, {7, 4}, {9, 9}, {20, 13}, {33, 33},
                              {64, 64}, {65, 64}, {100, 37}, {129, 128}, {200, 200}, {257, 131}, {300, 300}};
    const int tilings[][2] = {{6, 1}, {6, 2}, {6, 4}, {6, 8}, {12, 1}, {12, 3}, {12, 7}, {12, 15}, {18, 3}, {18, 7}};
    for (auto &s : shapes)
        for (auto &t : tilings)
            for (int threads : {64, 256, 1024}) {
                const int64_t m = s[0], n = s[1];
                const int k0 = t[0], nw = t[1];
                auto P = build_plan(m, n, k0, nw, threads);
                CHECK(P && P->m == m && P->n == n && P->K == k0 * nw);
                CHECK(P->N == (m == n ? n : n + 1));
                CHECK(P->L >= 64 && P->L <= threads && P->L % 64 == 0);
                int64_t rot[2] = {0, 0}, tend = 0;
                std::vector<int64_t> lane_end((size_t)P->L, 0);
                int folds = 0;
                for (size_t c = 0; c < P->chains.size(); ++c) {
                    const GenChain &g = P->chains[c];
                    CHECK(g.len >= 1 && g.tau0 >= 0);
                    // a thread runs chains c, c + L, ... one after another
                    CHECK(g.tau0 >= lane_end[c % (size_t)P->L]);
                    lane_end[c % (size_t)P->L] = g.tau0 + g.len;
                    tend = std::max<int64_t>(tend, g.tau0 + g.len);
                    if (g.type == CH_FOLD) {
                        ++folds;
                        continue;
                    }
                    for (int q = 0; q < g.len; ++q) {
                        const Rot r = decode(g.type, g.param, q);
                        CHECK(r.side == 0 || r.side == 1);
                        CHECK(r.i >= 1 && r.i <= (r.side == 0 ? P->N - 1 : n - 1));
                        ++rot[r.side];
                    }
                    for (int side = 0; side < 2; ++side)
                        if (g.slot[side] >= 0) CHECK(g.slot[side] < P->slots[side]);
                }
                CHECK(folds == 1);
                CHECK(rot[0] == P->nleft && rot[1] == P->nright);
                CHECK(tend == P->ticks);
                CHECK(P->split == 0 || (P->split > 0 && P->split < P->ticks));
                CHECK(P->nspike == (m > n ? m - n - 1 : 0));
                for (int side = 0; side < 2; ++side) {
                    CHECK((int)P->blocks[side].size() == P->nb1 + P->nb2);
                    int64_t pos = 0;
                    for (const BlockDesc &b : P->blocks[side]) {
                        CHECK(b.off == pos);
                        CHECK(b.nfront % (k0 + 3) == 0);
                        pos += (int64_t)b.nfront * P->K;
                    }
                    CHECK(pos == P->slots[side]);
                }
                CHECK(P->nseg >= 0 && P->nseg <= kMaxSeg);
                for (int k = 0; k < P->nseg; ++k) {
                    CHECK(P->tcut[k] > (k ? P->tcut[k - 1] : 0));
                    CHECK(P->bcut[k] > (k ? P->bcut[k - 1] : 0));
                }
                if (P->nseg > 0) {
                    CHECK(P->tcut[P->nseg - 1] == P->ticks);
                    CHECK(P->bcut[P->nseg - 1] == P->nb1 + P->nb2);
                }
            }
    if (g_fail) {
        fprintf(stderr, "%d checks failed\n", g_fail);
        return 1;
    }
    printf("plan: all checks passed\n");
    return 0;
}
