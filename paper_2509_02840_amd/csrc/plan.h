// plan.h -- host-side rotation schedule for one shape (m, n) and applier tiling.
#pragma once
#include <stdint.h>

#include <memory>
#include <vector>

#include "device.h"
#include "schedule.h"

namespace bdu {

struct Plan {
    int64_t m = 0, n = 0, N = 0;
    int K0 = 0, NW = 0, K = 0, S = 0;
    int L = 0;                      // generation threads
    std::vector<GenChain> chains;   // non-empty chains in schedule order (with the fold)
    std::vector<GenStart> starts;   // their first two rotations decoded (empty when the band
                                    // offsets exceed 16 bits, i.e. the band cannot be in LDS)
    int64_t ticks = 0;              // generation ticks
    int64_t split = 0;              // tick where phase 1 ends with nothing in flight (0: no split)
    int nseg = 0;                   // phase-2 segments (HandleDev::tcut, bcut)
    int32_t tcut[kMaxSeg] = {}, bcut[kMaxSeg] = {};
    int fold_seg = 0;               // the segment whose ticks include the fold
    int64_t nleft = 0, nright = 0;  // rotations of phases 1 and 2 per side
    int64_t nspike = 0;             // spike rotations (m > n)
    std::vector<BlockDesc> blocks[2];  // per side: phase-1 blocks, then phase-2 blocks
    int nb1 = 0, nb2 = 0;
    int64_t slots[2] = {0, 0};

    // device copies (owned by the plan cache, freed at unload)
    GenChain *d_chains = nullptr;
    GenStart *d_starts = nullptr;
    BlockDesc *d_blocks[2] = {nullptr, nullptr};
};

// Build (no device work).  gen_threads is the number of generation threads.
std::unique_ptr<Plan> build_plan(int64_t m, int64_t n, int K0, int NW, int gen_threads);

}  // namespace bdu
