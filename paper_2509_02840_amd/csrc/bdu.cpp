// bdu.cpp -- host side of the C ABI in include/bdu.h.
//
// A handle owns device copies of Q, d, e, P, the projection vectors, staging
// for update columns and the two rotation streams of its shape's schedule.
// Schedules (chains, generation ticks, applier blocks) are built once per
// (m, n, tiling) and shared by every handle of that shape.
#include "../../include/bdu.h"

#include <hip/hip_runtime.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <memory>
#include <mutex>
#include <initializer_list>
#include <set>
#include <tuple>
#include <vector>

#include "device.h"
#include "kernels.h"
#include "plan.h"
#include "bhu.h"
#include "orth.h"
#include "trbd.h"
#include "track.h"

using namespace bdu;

namespace {

std::mutex g_mu;
int g_k0 = 12, g_nw = 7, g_rpl = 1;  // 0, 0, 0: per-shape tuned tiling ("auto")
constexpr int kDefK0 = 12, kDefNW = 7, kDefRpl = 1;
struct Tuned {
    int k0, nw, rpl;
    double us;  // measured microseconds per batched step
};
std::map<std::pair<int64_t, int64_t>, Tuned> g_tuned;
bool g_gen_lds = true;  // generation keeps its band in LDS when it fits
bool g_check_finite = false;  // reject NaN / Inf inputs (one extra pass and a sync per call)
constexpr int64_t kSplitMinN = 32;  // smallest n whose single-handle passes split
bool g_split = true;          // single-handle passes apply phase 1 while phase 2 is generated
bool g_segments = true;       // ... and phase 2 in segments, each applied while the next is generated

struct PlanEntry {
    std::unique_ptr<Plan> plan;
    bool uploaded = false;
};
std::map<std::tuple<int64_t, int64_t, int, int>, PlanEntry> g_plans;

Plan *get_plan(int64_t m, int64_t n, int k0, int nw, bool upload, hipError_t *err)
{
    std::lock_guard<std::mutex> lk(g_mu);
    auto key = std::make_tuple(m, n, k0, nw);
    auto it = g_plans.find(key);
    if (it == g_plans.end()) {
        PlanEntry e;
        e.plan = build_plan(m, n, k0, nw, kGenThreads);
        it = g_plans.emplace(key, std::move(e)).first;
    }
    Plan *p = it->second.plan.get();
    if (upload && !it->second.uploaded) {
        size_t cb = sizeof(GenChain) * p->chains.size();
        hipError_t e = hipMalloc(&p->d_chains, cb);
        if (e == hipSuccess) e = hipMemcpy(p->d_chains, p->chains.data(), cb, hipMemcpyHostToDevice);
        if (e == hipSuccess && !p->starts.empty()) {
            size_t sb = sizeof(GenStart) * p->starts.size();
            e = hipMalloc(&p->d_starts, sb);
            if (e == hipSuccess) e = hipMemcpy(p->d_starts, p->starts.data(), sb, hipMemcpyHostToDevice);
        }
        for (int s = 0; s < 2 && e == hipSuccess; ++s) {
            size_t bb = sizeof(BlockDesc) * p->blocks[s].size();
            e = hipMalloc(&p->d_blocks[s], bb);
            if (e == hipSuccess) e = hipMemcpy(p->d_blocks[s], p->blocks[s].data(), bb, hipMemcpyHostToDevice);
        }
        if (e != hipSuccess) {
            *err = e;
            return nullptr;
        }
        it->second.uploaded = true;
    }
    *err = hipSuccess;
    return p;
}

bool is_device_ptr(const void *p)
{
    if (!p) return false;
    hipPointerAttribute_t a;
    hipError_t e = hipPointerGetAttributes(&a, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

// ---- stage timing --------------------------------------------------------
// When enabled, each kernel launch is bracketed by a pair of HIP events on
// the stream it runs on; reading sums the elapsed times per stage.
enum Stage { ST_PROJECT = 0, ST_SPIKE = 1, ST_GEN = 2, ST_APPLY = 3, ST_COUNT = 4 };
std::mutex g_tmu;
bool g_timing = false;
struct EvPair {
    int stage;
    hipEvent_t a, b;
};
std::vector<EvPair> g_events;
std::vector<hipEvent_t> g_pool;

hipEvent_t pool_get()
{
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

bool timing_on()
{
    std::lock_guard<std::mutex> lk(g_tmu);
    return g_timing;
}

// Launch `fn` as stage `stage` on stream st, timed when timing is on.
template <typename Fn>
hipError_t timed(int stage, hipStream_t st, Fn fn)
{
    bool on;
    {
        std::lock_guard<std::mutex> lk(g_tmu);
        on = g_timing;
    }
    if (!on) return fn();
    hipEvent_t a, b;
    {
        std::lock_guard<std::mutex> lk(g_tmu);
        a = pool_get();
        b = pool_get();
    }
    if (!a || !b) return fn();
    hipError_t e = hipEventRecord(a, st);
    if (e == hipSuccess) e = fn();
    if (e == hipSuccess) e = hipEventRecord(b, st);
    std::lock_guard<std::mutex> lk(g_tmu);
    g_events.push_back(EvPair{stage, a, b});
    return e;
}

}  // namespace

struct bdu_ctx {
    int64_t m = 0, n = 0;
    Plan *plan = nullptr;
    HandleDev hd{};
    HandleDev *d_hd = nullptr;
    HandleDev **d_self = nullptr;
    hipStream_t stream = nullptr;
    bool poisoned = false;
    int rcap = 0;
    int rpl = 1;  // rows per lane in the applier
    bool lds_gen = true;
    int *flag = nullptr;       // device flag of the non-finite input check
    hipEvent_t ev = nullptr;   // marks this handle's own stream work for a batch to wait on
    hipEvent_t dep = nullptr;  // completion of the last batch step this handle was in
    // split pass: phase 1 is applied on `side` while phase 2 is generated on
    // `stream`; sp1/sp2 mark the ends of the two generation parts, sp3 the
    // end of the application
    hipStream_t side = nullptr;
    hipEvent_t sp1 = nullptr, sp2 = nullptr, sp3 = nullptr;
    hipEvent_t seg[kMaxSeg] = {};  // ends of the phase-2 segments
    // orthogonality monitor scratch (allocated on first use)
    double *orthE = nullptr, *orthY = nullptr, *orthPart = nullptr, *orthOut = nullptr;
    // Householder update scratch (allocated on first use)
    double *bhu = nullptr;
    std::vector<void *> allocs;
};

namespace {

#define HIPCHK(h, expr)                      \
    do {                                     \
        hipError_t e_ = (expr);              \
        if (e_ != hipSuccess) {              \
            if (h) (h)->poisoned = true;     \
            return BDU_EDEVICE;              \
        }                                    \
    } while (0)

bool check_finite_on()
{
    std::lock_guard<std::mutex> lk(g_mu);
    return g_check_finite;
}

// With the check on: BDU_ENONFINITE if any value of the device ranges
// (pointer, count) is NaN or infinite, else BDU_OK (waits for the stream).
int check_finite(bdu_ctx *h, std::initializer_list<std::pair<const double *, int64_t>> ranges, hipStream_t st)
{
    if (!check_finite_on()) return BDU_OK;
    if (hipMemsetAsync(h->flag, 0, sizeof(int), st) != hipSuccess) return BDU_EDEVICE;
    for (auto &rg : ranges)
        if (launch_nonfinite(rg.first, rg.second, h->flag, st) != hipSuccess) return BDU_EDEVICE;
    int f = 0;
    if (hipMemcpyAsync(&f, h->flag, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return BDU_EDEVICE;
    return f ? BDU_ENONFINITE : BDU_OK;
}

// Order the handle's stream after the last batch step that updated it.
hipError_t wait_dep(bdu_ctx *h)
{
    return h->dep ? hipStreamWaitEvent(h->stream, h->dep, 0) : hipSuccess;
}

template <typename T>
hipError_t dalloc(bdu_ctx *h, T **p, int64_t count)
{
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, (size_t)std::max<int64_t>(count, 1) * sizeof(T));
    if (e == hipSuccess) {
        h->allocs.push_back(q);
        *p = (T *)q;
    }
    return e;
}

// Copy `bytes` from src (host or device) to the device buffer dst, in
// stream order.  Host sources are consumed before returning.
hipError_t copy_in(void *dst, const void *src, size_t bytes, hipStream_t st)
{
    if (bytes == 0) return hipSuccess;
    if (is_device_ptr(src)) return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st);
    hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(st);
}

// Column-major rows x cols matrix with leading dimension ld (doubles) on the
// device from a packed (leading dimension rows) host or device matrix.
hipError_t copy_mat_in(double *dst, int64_t ld, const double *src, int64_t rows, int64_t cols, hipStream_t st)
{
    bool dev = is_device_ptr(src);
    hipError_t e = hipMemcpy2DAsync(dst, sizeof(double) * ld, src, sizeof(double) * rows, sizeof(double) * rows,
                                    cols, dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st);
    if (e != hipSuccess || dev) return e;
    return hipStreamSynchronize(st);
}

hipError_t copy_mat_out(double *dst, const double *src, int64_t ld, int64_t rows, int64_t cols, hipStream_t st)
{
    if (!dst) return hipSuccess;
    hipMemcpyKind k = is_device_ptr(dst) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    hipError_t e = hipMemcpy2DAsync(dst, sizeof(double) * rows, src, sizeof(double) * ld, sizeof(double) * rows,
                                    cols, k, st);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(st);
}

hipError_t copy_out(void *dst, const void *src, size_t bytes, hipStream_t st)
{
    if (bytes == 0 || !dst) return hipSuccess;
    hipMemcpyKind k = is_device_ptr(dst) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    hipError_t e = hipMemcpyAsync(dst, src, bytes, k, st);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(st);
}

int ensure_rcap(bdu_ctx *h, int r)
{
    if (r <= h->rcap) return BDU_OK;
    int nr = std::max(r, 2 * h->rcap);
    double *nb = nullptr, *nc = nullptr;
    if (hipMalloc(&nb, sizeof(double) * h->m * nr) != hipSuccess) return BDU_ENOMEM;
    if (hipMalloc(&nc, sizeof(double) * h->n * nr) != hipSuccess) {
        (void)hipFree(nb);
        return BDU_ENOMEM;
    }
    HIPCHK(h, hipStreamSynchronize(h->stream));
    for (auto &p : h->allocs)
        if (p == h->hd.bst || p == h->hd.cst) {
            (void)hipFree(p);
            p = nullptr;
        }
    h->allocs.erase(std::remove(h->allocs.begin(), h->allocs.end(), nullptr), h->allocs.end());
    h->allocs.push_back(nb);
    h->allocs.push_back(nc);
    h->hd.bst = nb;
    h->hd.cst = nc;
    h->rcap = nr;
    HIPCHK(h, hipMemcpy(h->d_hd, &h->hd, sizeof(HandleDev), hipMemcpyHostToDevice));
    return BDU_OK;
}

// Rotation stages of one pass (spike, generation, application) for `count`
// handles listed in the device array hs (all with the same tiling).
hipError_t run_rotation_stages(HandleDev *const *hs, int count, bool any_spike, int64_t lds_bytes,
                               bool in_lds, int gen_threads, int max_panels, int k0, int nw, int rpl, Gate gate,
                               hipStream_t st)
{
    hipError_t e = hipSuccess;
    if (any_spike) e = timed(ST_SPIKE, st, [&] { return launch_spike(hs, count, gate, st); });
    if (e == hipSuccess)
        e = timed(ST_GEN, st, [&] { return launch_gen(hs, count, lds_bytes, in_lds, gen_threads, gate, st); });
    if (e == hipSuccess)
        e = timed(ST_APPLY, st, [&] { return launch_apply(hs, count, max_panels, k0, nw, rpl, gate, st); });
    return e;
}

// The same stages for passes that split after phase 1 (every listed handle's
// schedule has a split tick): phase 1 is applied on `sd` while phase 2 is
// generated on st, and st waits for the application.
//   st: [spike] gen 1 -> e1 -> gen 2 -> e2 ............ wait e3
//   sd:          wait e1 -> apply 1 -> wait e2 -> apply 2 -> e3
hipError_t run_split_stages(HandleDev *const *hs, int count, bool any_spike, int64_t lds_bytes, bool in_lds,
                            int gen_threads, int max_panels, int k0, int nw, int rpl, Gate gate, hipStream_t st,
                            hipStream_t sd, hipEvent_t e1, hipEvent_t e2, hipEvent_t e3)
{
    Gate g1 = gate, g2 = gate;
    g1.part = 1;
    g2.part = 2;
    hipError_t e = hipSuccess;
    if (any_spike) e = timed(ST_SPIKE, st, [&] { return launch_spike(hs, count, g1, st); });
    if (e == hipSuccess)
        e = timed(ST_GEN, st, [&] { return launch_gen(hs, count, lds_bytes, in_lds, gen_threads, g1, st); });
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess)
        e = timed(ST_GEN, st, [&] { return launch_gen(hs, count, lds_bytes, in_lds, gen_threads, g2, st); });
    if (e == hipSuccess) e = hipEventRecord(e2, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(sd, e1, 0);
    if (e == hipSuccess)
        e = timed(ST_APPLY, sd, [&] { return launch_apply(hs, count, max_panels, k0, nw, rpl, g1, sd); });
    if (e == hipSuccess) e = hipStreamWaitEvent(sd, e2, 0);
    if (e == hipSuccess)
        e = timed(ST_APPLY, sd, [&] { return launch_apply(hs, count, max_panels, k0, nw, rpl, g2, sd); });
    if (e == hipSuccess) e = hipEventRecord(e3, sd);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, e3, 0);
    return e;
}

// The stages of a pass in nseg segments (every listed handle's plan has
// that many): segment k's application on sd once its generation is done,
// the next segment's generation beside it; st waits for the application.
// With fold_seg > 0 (and the events spk_in, spk_out) the spike runs on sd
// beside the first segments' generation: phase 1 does not touch u beyond
// row N - 1, so only the segment holding the fold, which reads u_N (the
// spike's survivor), waits for it; the generator reloads u_N at the start
// of every later segment.  Segment 0's application, which applies the
// spike's rotations, follows it on sd.
hipError_t run_segment_stages(HandleDev *const *hs, int count, bool any_spike, int64_t lds_bytes, bool in_lds,
                              int gen_threads, int max_panels, int k0, int nw, int rpl, Gate gate, int nseg,
                              hipStream_t st, hipStream_t sd, const hipEvent_t *ev, hipEvent_t done,
                              int fold_seg = 0, hipEvent_t spk_in = nullptr, hipEvent_t spk_out = nullptr)
{
    hipError_t e = hipSuccess;
    Gate g0 = gate;
    g0.part = 3;
    const bool beside = any_spike && fold_seg > 0 && spk_in && spk_out;
    if (beside) {
        e = hipEventRecord(spk_in, st);  // the projections are done
        if (e == hipSuccess) e = hipStreamWaitEvent(sd, spk_in, 0);
        if (e == hipSuccess) e = timed(ST_SPIKE, sd, [&] { return launch_spike(hs, count, g0, sd); });
        if (e == hipSuccess) e = hipEventRecord(spk_out, sd);
    } else if (any_spike) {
        e = timed(ST_SPIKE, st, [&] { return launch_spike(hs, count, g0, st); });
    }
    for (int k = 0; k < nseg && e == hipSuccess; ++k) {
        Gate gk = gate;
        gk.part = 3 + k;
        if (beside && k == fold_seg) e = hipStreamWaitEvent(st, spk_out, 0);
        if (e == hipSuccess)
            e = timed(ST_GEN, st, [&] { return launch_gen(hs, count, lds_bytes, in_lds, gen_threads, gk, st); });
        if (e == hipSuccess) e = hipEventRecord(ev[k], st);
    }
    for (int k = 0; k < nseg && e == hipSuccess; ++k) {
        Gate gk = gate;
        gk.part = 3 + k;
        e = hipStreamWaitEvent(sd, ev[k], 0);
        if (e == hipSuccess)
            e = timed(ST_APPLY, sd, [&] { return launch_apply(hs, count, max_panels, k0, nw, rpl, gk, sd); });
    }
    if (e == hipSuccess) e = hipEventRecord(done, sd);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, done, 0);
    return e;
}

int tiles_of(const bdu_ctx *h) { return (int)((h->m + 63) / 64 + (h->n + 63) / 64); }
int panels_of(const bdu_ctx *h)
{
    const int64_t ph = 64 * h->rpl;
    return (int)((h->m + ph - 1) / ph + (h->n + ph - 1) / ph);
}

int pass_single(bdu_ctx *h, int pass, bool project, const double *xb = nullptr, const double *xc = nullptr)
{
    hipError_t e = hipSuccess;
    hipStream_t st = h->stream;
    if (project)
        e = timed(ST_PROJECT, st,
                  [&] { return launch_project(h->d_self, 1, tiles_of(h), Gate{nullptr, pass, 0, xb, xc}, st); });
    const int64_t lds = gen_lds_bytes(h->n, h->plan->N);
    const int L = h->plan->L, np = panels_of(h), k0 = h->plan->K0, nw = h->plan->NW;
    if (e == hipSuccess && h->side && h->plan->nseg > 0 && h->seg[0]) {
        // sp1 and sp2 (the split pass's events) order the spike beside the
        // generation
        e = run_segment_stages(h->d_self, 1, h->m > h->n, lds, h->lds_gen, L, np, k0, nw, h->rpl,
                               Gate{nullptr, pass, 0}, h->plan->nseg, st, h->side, h->seg, h->sp3,
                               h->plan->fold_seg, h->sp1, h->sp2);
    } else if (e == hipSuccess && h->side) {
        e = run_split_stages(h->d_self, 1, h->m > h->n, lds, h->lds_gen, L, np, k0, nw, h->rpl, Gate{nullptr, pass, 0},
                             st, h->side, h->sp1, h->sp2, h->sp3);
    } else if (e == hipSuccess) {
        e = run_rotation_stages(h->d_self, 1, h->m > h->n, lds, h->lds_gen, L, np, k0, nw, h->rpl,
                                Gate{nullptr, pass}, st);
    }
    if (e != hipSuccess) {
        h->poisoned = true;
        return BDU_EDEVICE;
    }
    return BDU_OK;
}

// Slot of a rotation in its side's stream (the layout the generator writes).
int64_t slot_of(const Plan &P, const GenChain &g, const Rot &r)
{
    const int ph = chain_phase(g.type), tg = chain_in_phase(g.type, g.param);
    const int b = tg / P.K, tin = tg % P.K, w = tin / P.K0, tl = tin % P.K0;
    const BlockDesc &bd = P.blocks[r.side][(ph == 1 ? 0 : P.nb1) + b];
    const int lam0 = lam0_of_pair(ph, bd.base, r.i);
    const int pos = front_order(2 * (ph - 1) + r.side, P.K, P.K0).pos[tl];
    return bd.off + (int64_t)(lam0 / 3 + tl + w * P.S) * P.K + w * P.K0 + pos;
}

}  // namespace

namespace {

bool segments_on()
{
    std::lock_guard<std::mutex> lk(g_mu);
    return g_segments;
}

bool split_on()
{
    std::lock_guard<std::mutex> lk(g_mu);
    return g_split;
}

void release_streams(bdu_ctx *h)
{
    if (h->ev) (void)hipEventDestroy(h->ev);
    if (h->sp1) (void)hipEventDestroy(h->sp1);
    if (h->sp2) (void)hipEventDestroy(h->sp2);
    if (h->sp3) (void)hipEventDestroy(h->sp3);
    for (int k = 0; k < kMaxSeg; ++k)
        if (h->seg[k]) (void)hipEventDestroy(h->seg[k]);
    if (h->side) (void)hipStreamDestroy(h->side);
    h->ev = h->sp1 = h->sp2 = h->sp3 = nullptr;
    for (int k = 0; k < kMaxSeg; ++k) h->seg[k] = nullptr;
    h->side = nullptr;
}

bool gen_lds_fits(int64_t n, int64_t N)
{
    std::lock_guard<std::mutex> lk(g_mu);
    return g_gen_lds && gen_lds_bytes(n, N) <= kMaxGenLds;
}

// Applier tiling for a new handle of shape (m, n).
void tiling_for(int64_t m, int64_t n, int *k0, int *nw, int *rpl)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_k0 != 0) {
        *k0 = g_k0;
        *nw = g_nw;
        *rpl = g_rpl;
        return;
    }
    auto it = g_tuned.find({m, n});
    if (it != g_tuned.end()) {
        *k0 = it->second.k0;
        *nw = it->second.nw;
        *rpl = it->second.rpl;
    } else {
        *k0 = kDefK0;
        *nw = kDefNW;
        *rpl = kDefRpl;
    }
}

int create_impl(int64_t m, int64_t n, const double *Q, const double *d, const double *e, const double *P, int k0,
                int nw, int rpl, bdu_handle *out);

}  // namespace

// A fixed set of distinct handles updated together (see bdu_batch_create).
struct bdu_batch_ctx {
    std::vector<bdu_ctx *> hs;  // caller's order
    std::vector<int> pos;       // position of hs[i] in the launch arrays
    int maxr = 1;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    struct Group {
        int k0, nw, rpl;
        bool spike, in_lds;
        int64_t lds;
        int tiles, panels, off, cnt;
        int gen_threads;  // largest plan thread count of the group
        bool split;       // every member's pass splits after phase 1
        int nseg;         // segments of the group: the largest member's count (0: no segments)
    };
    std::vector<Group> groups;  // handles of one applier tiling, contiguous in the arrays
    HandleDev **d_ptrs = nullptr;
    int32_t *d_ranks = nullptr;
    int32_t *h_ranks = nullptr;  // pinned staging of the ranks
    hipEvent_t ranks_copied = nullptr, done = nullptr;
    hipEvent_t null_ready = nullptr;  // own stream: the null stream's work before a step
    // split passes: phase 1 applied on `side` while phase 2 is generated
    hipStream_t side = nullptr;
    hipEvent_t sp1 = nullptr, sp2 = nullptr, sp3 = nullptr;
    hipEvent_t seg[kMaxSeg] = {};
    bool use_graph = false;
    int64_t steps = 0;
    hipGraphExec_t exec = nullptr;
    bool poisoned = false;
};

namespace {

void batch_free(bdu_batch b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->d_ptrs) (void)hipFree(b->d_ptrs);
    if (b->d_ranks) (void)hipFree(b->d_ranks);
    if (b->h_ranks) (void)hipHostFree(b->h_ranks);
    if (b->ranks_copied) (void)hipEventDestroy(b->ranks_copied);
    if (b->done) (void)hipEventDestroy(b->done);
    if (b->null_ready) (void)hipEventDestroy(b->null_ready);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    if (b->sp1) (void)hipEventDestroy(b->sp1);
    if (b->sp2) (void)hipEventDestroy(b->sp2);
    if (b->sp3) (void)hipEventDestroy(b->sp3);
    for (int k = 0; k < kMaxSeg; ++k)
        if (b->seg[k]) (void)hipEventDestroy(b->seg[k]);
    if (b->side) (void)hipStreamDestroy(b->side);
    delete b;
}

int batch_build(const bdu_handle *hs, int count, int maxr, bool graph, bdu_batch *out)
{
    if (!hs || count < 1 || maxr < 1) return BDU_EINVAL;
    std::set<bdu_ctx *> seen;
    for (int i = 0; i < count; ++i) {
        if (!hs[i] || !seen.insert(hs[i]).second) return BDU_EINVAL;  // NULL or repeated handle
        if (hs[i]->poisoned) return BDU_EDEVICE;
    }
    for (int i = 0; i < count; ++i) {
        int s = ensure_rcap(hs[i], maxr);
        if (s != BDU_OK) return s;
    }
    auto b = new bdu_batch_ctx;
    b->hs.assign(hs, hs + count);
    b->maxr = maxr;
    b->use_graph = graph;
    hipError_t e = hipSuccess;
    if (graph) {
        // non-blocking: a graph is captured on it, and capture on a stream
        // that synchronizes implicitly with the null stream would fail the
        // null-stream work of any other thread meanwhile
        e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
        b->own_stream = e == hipSuccess;
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->null_ready, hipEventDisableTiming);
    } else {
        b->stream = hs[0]->stream;
    }
    // group by tiling (and generation placement)
    std::vector<std::vector<int>> members;
    for (int i = 0; i < count; ++i) {
        bdu_ctx *h = hs[i];
        size_t g = 0;
        for (; g < b->groups.size(); ++g) {
            auto &x = b->groups[g];
            if (x.k0 == h->plan->K0 && x.nw == h->plan->NW && x.rpl == h->rpl && x.in_lds == h->lds_gen) break;
        }
        if (g == b->groups.size()) {
            b->groups.push_back({h->plan->K0, h->plan->NW, h->rpl, false, h->lds_gen, 0, 0, 0, 0, 0, 64, split_on(),
                                 segments_on() ? h->plan->nseg : 0});
            members.emplace_back();
        }
        auto &x = b->groups[g];
        members[g].push_back(i);
        x.spike |= h->m > h->n;
        x.lds = std::max<int64_t>(x.lds, gen_lds_bytes(h->n, h->plan->N));
        x.gen_threads = std::max(x.gen_threads, h->plan->L);
        x.tiles = std::max(x.tiles, tiles_of(h));
        x.panels = std::max(x.panels, panels_of(h));
        x.split = x.split && h->plan->split > 0;
        // the group runs as many segments as its largest plan has (the
        // kernels skip a handle's segments past its own count)
        if (x.nseg > 0) x.nseg = segments_on() && h->plan->nseg > 0 ? std::max(x.nseg, h->plan->nseg) : 0;
    }
    bool any_split = false;
    int max_seg = 0;
    for (auto &x : b->groups) {
        any_split |= x.split || x.nseg > 0;
        max_seg = std::max(max_seg, x.nseg);
    }
    std::vector<HandleDev *> flat;
    b->pos.assign(count, 0);
    for (size_t g = 0; g < b->groups.size(); ++g) {
        b->groups[g].off = (int)flat.size();
        b->groups[g].cnt = (int)members[g].size();
        for (int i : members[g]) {
            b->pos[i] = (int)flat.size();
            flat.push_back(hs[i]->d_hd);
        }
    }
    if (e == hipSuccess) e = hipMalloc(&b->d_ptrs, sizeof(HandleDev *) * count);
    if (e == hipSuccess) e = hipMalloc(&b->d_ranks, sizeof(int32_t) * count);
    if (e == hipSuccess) e = hipHostMalloc(&b->h_ranks, sizeof(int32_t) * count, hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ranks_copied, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->done, hipEventDisableTiming);
    if (e == hipSuccess && any_split) {
        e = hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->sp1, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->sp2, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->sp3, hipEventDisableTiming);
        for (int k = 0; e == hipSuccess && k < max_seg; ++k)
            e = hipEventCreateWithFlags(&b->seg[k], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = prepare_kernels();
    if (e == hipSuccess) e = hipMemcpy(b->d_ptrs, flat.data(), sizeof(HandleDev *) * count, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        batch_free(b);
        return e == hipErrorOutOfMemory ? BDU_ENOMEM : BDU_EDEVICE;
    }
    *out = b;
    return BDU_OK;
}

// One step's launches: for each pass, every tiling group (handles whose rank
// this step is at most the pass leave at once).
hipError_t batch_launch(bdu_batch b)
{
    hipStream_t st = b->stream;
    for (int p = 0; p < b->maxr; ++p) {
        for (auto &g : b->groups) {
            HandleDev **arr = b->d_ptrs + g.off;
            const Gate gate{b->d_ranks + g.off, p};
            hipError_t e = timed(ST_PROJECT, st, [&] { return launch_project(arr, g.cnt, g.tiles, gate, st); });
            if (e == hipSuccess && g.nseg > 0 && b->side)
                e = run_segment_stages(arr, g.cnt, g.spike, g.lds, g.in_lds, g.gen_threads, g.panels, g.k0, g.nw,
                                       g.rpl, gate, g.nseg, st, b->side, b->seg, b->sp3);
            else if (e == hipSuccess && g.split && b->side)
                e = run_split_stages(arr, g.cnt, g.spike, g.lds, g.in_lds, g.gen_threads, g.panels, g.k0, g.nw,
                                     g.rpl, gate, st, b->side, b->sp1, b->sp2, b->sp3);
            else if (e == hipSuccess)
                e = run_rotation_stages(arr, g.cnt, g.spike, g.lds, g.in_lds, g.gen_threads, g.panels, g.k0, g.nw,
                                        g.rpl, gate, st);
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

}  // namespace

extern "C" {

const char *bdu_strerror(int status)
{
    switch (status) {
    case BDU_OK: return "ok";
    case BDU_EINVAL: return "invalid argument";
    case BDU_ENOMEM: return "out of device memory";
    case BDU_EDEVICE: return "device error (handle poisoned)";
    case BDU_ENONFINITE: return "non-finite input";
    case BDU_EBUSY: return "queue full";
    case BDU_ESPAN: return "rank-1 tracker with an update vector in the span of its basis";
    case BDU_ESCRATCH: return "update larger than the no-allocation scratch (bdu_noalloc_capacity)";
    default: return "unknown status";
    }
}

int bdu_set_tiling(int k0, int nw, int rpl)
{
    if (!(k0 == 0 && nw == 0 && rpl == 0) && !tiling_supported(k0, nw, rpl)) return BDU_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    g_k0 = k0;
    g_nw = nw;
    g_rpl = rpl;
    return BDU_OK;
}

int bdu_get_tiling(int *k0, int *nw, int *rpl)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (k0) *k0 = g_k0;
    if (nw) *nw = g_nw;
    if (rpl) *rpl = g_rpl;
    return BDU_OK;
}

int64_t bdu_footprint_bytes(int64_t m, int64_t n)
{
    if (m < n || n < 2) return BDU_EINVAL;
    int k0, nw, rpl;
    tiling_for(m, n, &k0, &nw, &rpl);
    hipError_t e;
    Plan *p = get_plan(m, n, k0, nw, false, &e);
    int64_t N = p->N;
    const int64_t ldq = (m + 127) / 128 * 128, ldp = (n + 127) / 128 * 128;
    int64_t bytes = 8 * (ldq * m + ldp * n + 2 * n + 2 * (m + n) + 2 * (m + n));
    bytes += 16 * (p->slots[0] + p->slots[1] + 2 * (4 * (int64_t)p->K + 64) + std::max<int64_t>(p->nspike, 1));
    bytes += gen_lds_bytes(n, N);  // band (device memory or the image between split parts)
    return bytes;
}

int bdu_create(int64_t m, int64_t n, const double *Q, const double *d, const double *e, const double *P,
               bdu_handle *out)
{
    if (!out || !Q || !d || !e || !P || m < n || n < 2 || m > (int64_t)1 << 30) return BDU_EINVAL;
    *out = nullptr;
    int k0, nw, rpl;
    tiling_for(m, n, &k0, &nw, &rpl);
    return create_impl(m, n, Q, d, e, P, k0, nw, rpl, out);
}

int bdu_set_finite_check(int on)
{
    if (on != 0 && on != 1) return BDU_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    g_check_finite = on != 0;
    return BDU_OK;
}

int bdu_set_generation_in_lds(int allow)
{
    if (allow != 0 && allow != 1) return BDU_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    g_gen_lds = allow != 0;
    return BDU_OK;
}

int bdu_set_split_pass(int on)
{
    if (on < 0 || on > 2) return BDU_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    g_split = on != 0;
    g_segments = on == 2;
    return BDU_OK;
}

int bdu_handle_tiling(bdu_handle h, int *k0, int *nw, int *rpl)
{
    if (!h) return BDU_EINVAL;
    if (k0) *k0 = h->plan->K0;
    if (nw) *nw = h->plan->NW;
    if (rpl) *rpl = h->rpl;
    return BDU_OK;
}

}  // extern "C"

namespace {

int create_impl(int64_t m, int64_t n, const double *Q, const double *d, const double *e, const double *P, int k0,
                int nw, int rpl, bdu_handle *out)
{
    hipError_t err;
    Plan *plan = get_plan(m, n, k0, nw, true, &err);
    if (!plan) return BDU_EDEVICE;
    auto h = std::make_unique<bdu_ctx>();
    h->m = m;
    h->n = n;
    h->plan = plan;
    h->rpl = rpl;
    h->lds_gen = gen_lds_fits(n, plan->N);
    HandleDev &hd = h->hd;
    hipError_t a = hipSuccess;
    auto A = [&](hipError_t x) { if (a == hipSuccess) a = x; };
    const int64_t ldq = (m + 127) / 128 * 128, ldp = (n + 127) / 128 * 128;
    A(dalloc(h.get(), &hd.Q, ldq * m));
    A(dalloc(h.get(), &hd.P, ldp * n));
    A(dalloc(h.get(), &hd.d, n));
    A(dalloc(h.get(), &hd.e, n));
    A(dalloc(h.get(), &hd.u, m));
    A(dalloc(h.get(), &hd.v, n));
    A(dalloc(h.get(), &hd.bst, m));
    A(dalloc(h.get(), &hd.cst, n));
    // slack of a few fronts: the applier releases the address of the next
    // front's coefficients one group early, also after a block's last front
    const int64_t slack = 4 * (int64_t)plan->K + 64;
    A(dalloc(h.get(), &hd.csL, plan->slots[0] + slack));
    A(dalloc(h.get(), &hd.csR, plan->slots[1] + slack));
    A(dalloc(h.get(), &hd.csSp, plan->nspike));
    // the band in device memory (large n), or the image of the LDS band
    // kept between the two parts of a split generation
    A(dalloc(h.get(), &hd.band, gen_lds_bytes(n, plan->N) / 8));
    A(dalloc(h.get(), &hd.carry, 4 * kGenThreads));
    A(dalloc(h.get(), &h->d_hd, 1));
    A(dalloc(h.get(), &h->d_self, 1));
    A(dalloc(h.get(), &h->flag, 1));
    if (a != hipSuccess) {
        for (void *p : h->allocs) (void)hipFree(p);
        (void)hipGetLastError();
        return BDU_ENOMEM;
    }
    h->rcap = 1;
    hd.chains = plan->d_chains;
    hd.starts = plan->d_starts;
    hd.blkL = plan->d_blocks[0];
    hd.blkR = plan->d_blocks[1];
    hd.ticks = plan->ticks;
    hd.split = plan->split;
    hd.nseg = plan->nseg;
    for (int k = 0; k < kMaxSeg; ++k) {
        hd.tcut[k] = plan->tcut[k];
        hd.bcut[k] = plan->bcut[k];
    }
    hd.m = (int32_t)m;
    hd.n = (int32_t)n;
    hd.ldq = (int32_t)ldq;
    hd.ldp = (int32_t)ldp;
    hd.N = (int32_t)plan->N;
    hd.nchains = (int32_t)plan->chains.size();
    hd.nb1 = plan->nb1;
    hd.nb2 = plan->nb2;
    hd.K0 = plan->K0;
    hd.NW = plan->NW;
    hd.K = plan->K;
    hd.S = plan->S;
    bdu_ctx *hp = h.get();
    HIPCHK(hp, hipMemsetAsync(hd.Q, 0, sizeof(double) * ldq * m, hp->stream));
    HIPCHK(hp, hipMemsetAsync(hd.P, 0, sizeof(double) * ldp * n, hp->stream));
    HIPCHK(hp, copy_mat_in(hd.Q, ldq, Q, m, m, hp->stream));
    HIPCHK(hp, copy_mat_in(hd.P, ldp, P, n, n, hp->stream));
    HIPCHK(hp, copy_in(hd.d, d, sizeof(double) * n, hp->stream));
    HIPCHK(hp, copy_in(hd.e, e, sizeof(double) * (n - 1), hp->stream));
    {
        const int fin = check_finite(hp, {{hd.Q, ldq * m}, {hd.P, ldp * n}, {hd.d, n}, {hd.e, n - 1}}, hp->stream);
        if (fin != BDU_OK) {
            (void)hipStreamSynchronize(hp->stream);
            for (void *p : hp->allocs) (void)hipFree(p);
            return fin;
        }
    }
    HIPCHK(hp, launch_fill_identity(hd.csL, plan->slots[0] + slack, hp->stream));
    HIPCHK(hp, launch_fill_identity(hd.csR, plan->slots[1] + slack, hp->stream));
    HIPCHK(hp, hipMemcpyAsync(h->d_hd, &hd, sizeof(HandleDev), hipMemcpyHostToDevice, hp->stream));
    HandleDev *self = h->d_hd;
    HIPCHK(hp, hipMemcpyAsync(h->d_self, &self, sizeof(self), hipMemcpyHostToDevice, hp->stream));
    HIPCHK(hp, hipStreamSynchronize(hp->stream));
    bool ok = hipEventCreateWithFlags(&hp->ev, hipEventDisableTiming) == hipSuccess;
    // below n = 32 a pass is a few hundred microseconds at most and the
    // second stream's event waits cost about what the overlap saves
    if (ok && plan->split > 0 && split_on() && n >= kSplitMinN) {
        ok = hipStreamCreateWithFlags(&hp->side, hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&hp->sp1, hipEventDisableTiming) == hipSuccess &&
             hipEventCreateWithFlags(&hp->sp2, hipEventDisableTiming) == hipSuccess &&
             hipEventCreateWithFlags(&hp->sp3, hipEventDisableTiming) == hipSuccess;
        for (int k = 0; ok && segments_on() && k < plan->nseg; ++k)
            ok = hipEventCreateWithFlags(&hp->seg[k], hipEventDisableTiming) == hipSuccess;
    }
    if (!ok) {
        release_streams(hp);
        for (void *p : h->allocs) (void)hipFree(p);
        return BDU_EDEVICE;
    }
    *out = h.release();
    return BDU_OK;
}

}  // namespace

extern "C" {

int bdu_set_stream(bdu_handle h, void *stream)
{
    if (!h) return BDU_EINVAL;
    if (h->poisoned) return BDU_EDEVICE;
    HIPCHK(h, wait_dep(h));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    h->stream = (hipStream_t)stream;
    return BDU_OK;
}

int bdu_sync(bdu_handle h)
{
    if (!h) return BDU_EINVAL;
    if (h->poisoned) return BDU_EDEVICE;
    HIPCHK(h, wait_dep(h));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return BDU_OK;
}

int bdu_update(bdu_handle h, const double *B, const double *C, int r)
{
    if (!h || !B || !C || r < 1) return BDU_EINVAL;
    if (h->poisoned) return BDU_EDEVICE;
    HIPCHK(h, wait_dep(h));
    int st = ensure_rcap(h, r);
    if (st != BDU_OK) return st;
    HIPCHK(h, copy_in(h->hd.bst, B, sizeof(double) * h->m * r, h->stream));
    HIPCHK(h, copy_in(h->hd.cst, C, sizeof(double) * h->n * r, h->stream));
    st = check_finite(h, {{h->hd.bst, h->m * r}, {h->hd.cst, h->n * r}}, h->stream);
    if (st != BDU_OK) return st;
    for (int p = 0; p < r; ++p) {
        st = pass_single(h, p, true);
        if (st != BDU_OK) return st;
    }
    return BDU_OK;
}

// ---- update without allocation -----------------------------------------------
//
// bdu_update_noalloc stages B and C in a fixed device array instead of the
// handle's staging buffers, which bdu_update grows with hipMalloc when r
// exceeds their capacity.  In host code `scratch` names a host-side stand-in
// of the array; its device address is looked up once per device with
// hipGetSymbolAddress, and only that address is ever given to the runtime
// or a kernel.

}  // extern "C"

namespace {

constexpr int64_t kScratchDoubles = (int64_t)1 << 20;  // 8 MiB per device
static __device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_scratch_mu;
std::map<int, double *> g_scratch_ptr;  // device ordinal -> address of scratch

// The current device's copy of scratch (looked up on the first call there).
int scratch_ptr(double **out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return BDU_EDEVICE;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it == g_scratch_ptr.end()) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return BDU_EDEVICE;
        it = g_scratch_ptr.emplace(dev, (double *)p).first;
    }
    *out = it->second;
    return BDU_OK;
}

}  // namespace

extern "C" {

int64_t bdu_noalloc_capacity(void) { return kScratchDoubles; }

int bdu_update_noalloc(bdu_handle h, const double *B, const double *C, int r)
{
    if (!h || !B || !C || r < 1) return BDU_EINVAL;
    if (h->poisoned) return BDU_EDEVICE;
    if ((int64_t)r * (h->m + h->n) > kScratchDoubles) return BDU_ESCRATCH;
    double *xs = nullptr;
    int st = scratch_ptr(&xs);
    if (st != BDU_OK) return st;
    HIPCHK(h, wait_dep(h));
    double *xb = xs, *xc = xs + h->m * r;
    HIPCHK(h, copy_in(xb, B, sizeof(double) * h->m * r, h->stream));
    HIPCHK(h, copy_in(xc, C, sizeof(double) * h->n * r, h->stream));
    st = check_finite(h, {{xb, h->m * r}, {xc, h->n * r}}, h->stream);
    if (st != BDU_OK) return st;
    for (int p = 0; p < r; ++p) {
        st = pass_single(h, p, true, xb, xc);
        if (st != BDU_OK) return st;
    }
    return BDU_OK;
}

int bdu_update_projected(bdu_handle h, const double *u, const double *v)
{
    if (!h || !u || !v) return BDU_EINVAL;
    if (h->poisoned) return BDU_EDEVICE;
    HIPCHK(h, wait_dep(h));
    HIPCHK(h, copy_in(h->hd.u, u, sizeof(double) * h->m, h->stream));
    HIPCHK(h, copy_in(h->hd.v, v, sizeof(double) * h->n, h->stream));
    const int st = check_finite(h, {{h->hd.u, h->m}, {h->hd.v, h->n}}, h->stream);
    if (st != BDU_OK) return st;
    return pass_single(h, 0, false);
}

int bdu_project(bdu_handle h, const double *b, const double *c, double *u, double *v)
{
    if (!h || !b || !c) return BDU_EINVAL;
    if (h->poisoned) return BDU_EDEVICE;
    HIPCHK(h, wait_dep(h));
    HIPCHK(h, copy_in(h->hd.bst, b, sizeof(double) * h->m, h->stream));
    HIPCHK(h, copy_in(h->hd.cst, c, sizeof(double) * h->n, h->stream));
    HIPCHK(h, launch_project(h->d_self, 1, tiles_of(h), Gate{nullptr, 0}, h->stream));
    HIPCHK(h, copy_out(u, h->hd.u, sizeof(double) * h->m, h->stream));
    HIPCHK(h, copy_out(v, h->hd.v, sizeof(double) * h->n, h->stream));
    return BDU_OK;
}

int bdu_read(bdu_handle h, double *Q, double *d, double *e, double *P)
{
    if (!h) return BDU_EINVAL;
    if (h->poisoned) return BDU_EDEVICE;
    HIPCHK(h, wait_dep(h));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    HIPCHK(h, copy_mat_out(Q, h->hd.Q, h->hd.ldq, h->m, h->m, h->stream));
    HIPCHK(h, copy_out(d, h->hd.d, sizeof(double) * h->n, h->stream));
    HIPCHK(h, copy_out(e, h->hd.e, sizeof(double) * (h->n - 1), h->stream));
    HIPCHK(h, copy_mat_out(P, h->hd.P, h->hd.ldp, h->n, h->n, h->stream));
    return BDU_OK;
}

int64_t bdu_last_rotations(bdu_handle h, int32_t *side, int64_t *idx, double *c, double *s, int64_t cap)
{
    if (!h) return BDU_EINVAL;
    if (h->poisoned) return BDU_EDEVICE;
    HIPCHK(h, wait_dep(h));
    const Plan &P = *h->plan;
    std::vector<double2> L(P.slots[0]), R(P.slots[1]), Sp(std::max<int64_t>(P.nspike, 1));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    HIPCHK(h, hipMemcpy(L.data(), h->hd.csL, sizeof(double2) * P.slots[0], hipMemcpyDeviceToHost));
    HIPCHK(h, hipMemcpy(R.data(), h->hd.csR, sizeof(double2) * P.slots[1], hipMemcpyDeviceToHost));
    if (P.nspike) HIPCHK(h, hipMemcpy(Sp.data(), h->hd.csSp, sizeof(double2) * P.nspike, hipMemcpyDeviceToHost));
    int64_t k = 0;
    auto emit = [&](int sd, int64_t i, double2 v) {
        if (k < cap) {
            if (side) side[k] = sd;
            if (idx) idx[k] = i;
            if (c) c[k] = v.x;
            if (s) s[k] = v.y;
        }
        ++k;
    };
    for (int64_t t = 0; t < P.nspike; ++t) emit(0, P.m - 1 - t, Sp[t]);
    for (const GenChain &g : P.chains) {
        if (g.type == CH_FOLD) continue;
        for (int q = 0; q < g.len; ++q) {
            Rot r = decode(g.type, g.param, q);
            int64_t sl = slot_of(P, g, r);
            if (sl != g.slot[r.side] + (int64_t)(q >> 1) * P.K) return BDU_EDEVICE;  // layout invariant
            emit(r.side, r.i, r.side == 0 ? L[sl] : R[sl]);
        }
    }
    return k;
}

int bdu_destroy(bdu_handle h)
{
    if (!h) return BDU_EINVAL;
    (void)wait_dep(h);
    (void)hipStreamSynchronize(h->stream);
    if (h->side) (void)hipStreamSynchronize(h->side);
    for (void *p : h->allocs) (void)hipFree(p);
    release_streams(h);
    delete h;
    return BDU_OK;
}

int bdu_update_batched(const bdu_handle *hs, const double *const *Bs, const double *const *Cs, const int *rs,
                       int count)
{
    if (!hs || !Bs || !Cs || !rs || count < 1) return BDU_EINVAL;
    int maxr = 0;
    for (int i = 0; i < count; ++i) {
        if (rs[i] < 1) return BDU_EINVAL;
        maxr = std::max(maxr, rs[i]);
    }
    bdu_batch b = nullptr;
    int st = batch_build(hs, count, maxr, false, &b);
    if (st != BDU_OK) return st;
    st = bdu_batch_update(b, Bs, Cs, rs);
    if (st == BDU_OK) st = bdu_batch_sync(b);
    int st2 = bdu_batch_destroy(b);
    return st != BDU_OK ? st : st2;
}

int bdu_batch_create(const bdu_handle *hs, int count, int max_rank, bdu_batch *out)
{
    if (!out) return BDU_EINVAL;
    *out = nullptr;
    return batch_build(hs, count, max_rank, true, out);
}

int bdu_batch_create_flags(const bdu_handle *hs, int count, int max_rank, int flags, bdu_batch *out)
{
    if (!out || (flags & ~BDU_BATCH_EAGER)) return BDU_EINVAL;
    *out = nullptr;
    return batch_build(hs, count, max_rank, !(flags & BDU_BATCH_EAGER), out);
}

int bdu_batch_update(bdu_batch b, const double *const *Bs, const double *const *Cs, const int *rs)
{
    if (!b || !rs) return BDU_EINVAL;
    if (b->poisoned) return BDU_EDEVICE;
    const int count = (int)b->hs.size();
    for (int i = 0; i < count; ++i) {
        if (rs[i] < 0 || rs[i] > b->maxr) return BDU_EINVAL;
        if (rs[i] > 0 && (!Bs || !Cs || !Bs[i] || !Cs[i])) return BDU_EINVAL;
        if (b->hs[i]->poisoned) return BDU_EDEVICE;
    }
    hipStream_t st = b->stream;
    auto fail = [&]() {
        b->poisoned = true;
        for (bdu_ctx *h : b->hs) h->poisoned = true;
        return BDU_EDEVICE;
    };
    // the batch's own stream is ordered after the null stream's earlier
    // work explicitly (it does not synchronize with it implicitly)
    if (b->own_stream &&
        (hipEventRecord(b->null_ready, nullptr) != hipSuccess || hipStreamWaitEvent(st, b->null_ready, 0) != hipSuccess))
        return fail();
    // inputs, in stream order after each handle's own work
    for (int i = 0; i < count; ++i) {
        bdu_ctx *h = b->hs[i];
        if (h->stream != st) {
            if (hipEventRecord(h->ev, h->stream) != hipSuccess || hipStreamWaitEvent(st, h->ev, 0) != hipSuccess)
                return fail();
        }
        if (rs[i] == 0) continue;
        if (copy_in(h->hd.bst, Bs[i], sizeof(double) * h->m * rs[i], st) != hipSuccess ||
            copy_in(h->hd.cst, Cs[i], sizeof(double) * h->n * rs[i], st) != hipSuccess)
            return fail();
    }
    // non-finite inputs reject the whole step before any handle changes
    for (int i = 0; i < count; ++i) {
        if (rs[i] == 0) continue;
        bdu_ctx *h = b->hs[i];
        const int fin = check_finite(h, {{h->hd.bst, h->m * rs[i]}, {h->hd.cst, h->n * rs[i]}}, st);
        if (fin == BDU_ENONFINITE) return fin;
        if (fin != BDU_OK) return fail();
    }
    // this step's ranks (the pinned staging is reused once the last copy is done)
    if (b->steps > 0 && hipEventSynchronize(b->ranks_copied) != hipSuccess) return fail();
    for (int i = 0; i < count; ++i) b->h_ranks[b->pos[i]] = rs[i];
    if (hipMemcpyAsync(b->d_ranks, b->h_ranks, sizeof(int32_t) * count, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipEventRecord(b->ranks_copied, st) != hipSuccess)
        return fail();
    hipError_t e = hipSuccess;
    const bool graph_now = b->use_graph && !timing_on() && b->steps > 0;
    if (graph_now && !b->exec) {
        // capture one step's launches once; every later step replays them
        e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t el = batch_launch(b);
            hipGraph_t g = nullptr;
            e = hipStreamEndCapture(st, &g);
            if (el != hipSuccess) e = el;
            if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
            if (g) (void)hipGraphDestroy(g);
        }
        if (e != hipSuccess) return fail();
    }
    e = graph_now ? hipGraphLaunch(b->exec, st) : batch_launch(b);
    if (e != hipSuccess || hipEventRecord(b->done, st) != hipSuccess) return fail();
    for (bdu_ctx *h : b->hs) h->dep = b->done;
    ++b->steps;
    return BDU_OK;
}

int bdu_batch_sync(bdu_batch b)
{
    if (!b) return BDU_EINVAL;
    if (b->poisoned) return BDU_EDEVICE;
    if (hipStreamSynchronize(b->stream) != hipSuccess) {
        b->poisoned = true;
        return BDU_EDEVICE;
    }
    return BDU_OK;
}

int bdu_batch_info(bdu_batch b, int64_t *out)
{
    if (!b || !out) return BDU_EINVAL;
    out[0] = (int64_t)b->hs.size();
    out[1] = b->maxr;
    out[2] = (int64_t)b->groups.size();
    out[3] = b->exec != nullptr;
    out[4] = b->steps;
    return BDU_OK;
}

int bdu_batch_destroy(bdu_batch b)
{
    if (!b) return BDU_EINVAL;
    (void)hipStreamSynchronize(b->stream);
    for (bdu_ctx *h : b->hs)
        if (h->dep == b->done) h->dep = nullptr;
    batch_free(b);
    return BDU_OK;
}

int bdu_autotune(int64_t m, int64_t n, int streams, int64_t *out)
{
    if (m < n || n < 2 || streams < 1 || streams > 4096 || m > (int64_t)1 << 30) return BDU_EINVAL;
    // Synthetic streams: Q = I, P = I, d = 1, e = 1/2; every stream takes the
    // same update.  The applier's work does not depend on the values.
    double *dQ = nullptr, *dP = nullptr, *dd = nullptr, *de = nullptr, *db = nullptr, *dc = nullptr;
    hipStream_t st0 = nullptr;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    auto release = [&]() {
        for (double *p : {dQ, dP, dd, de, db, dc})
            if (p) (void)hipFree(p);
        if (t0) (void)hipEventDestroy(t0);
        if (t1) (void)hipEventDestroy(t1);
    };
    hipError_t e = hipSuccess;
    auto A = [&](hipError_t x) { if (e == hipSuccess) e = x; };
    A(hipMalloc(&dQ, sizeof(double) * m * m));
    A(hipMalloc(&dP, sizeof(double) * n * n));
    A(hipMalloc(&dd, sizeof(double) * n));
    A(hipMalloc(&de, sizeof(double) * n));
    A(hipMalloc(&db, sizeof(double) * m));
    A(hipMalloc(&dc, sizeof(double) * n));
    A(hipEventCreate(&t0));
    A(hipEventCreate(&t1));
    if (e != hipSuccess) {
        release();
        (void)hipGetLastError();
        return e == hipErrorOutOfMemory ? BDU_ENOMEM : BDU_EDEVICE;
    }
    std::vector<double> ones(m, 1.0), half(n, 0.5), bv(m), cv(n);
    for (int64_t i = 0; i < m; ++i) bv[i] = ((i * 7919) % 1000) / 1000.0 - 0.5;
    for (int64_t i = 0; i < n; ++i) cv[i] = ((i * 104729) % 1000) / 1000.0 - 0.5;
    A(hipMemset(dQ, 0, sizeof(double) * m * m));
    A(hipMemset(dP, 0, sizeof(double) * n * n));
    A(hipMemcpy2D(dQ, sizeof(double) * (m + 1), ones.data(), sizeof(double), sizeof(double), m,
                  hipMemcpyHostToDevice));
    A(hipMemcpy2D(dP, sizeof(double) * (n + 1), ones.data(), sizeof(double), sizeof(double), n,
                  hipMemcpyHostToDevice));
    A(hipMemcpy(dd, ones.data(), sizeof(double) * n, hipMemcpyHostToDevice));
    A(hipMemcpy(de, half.data(), sizeof(double) * n, hipMemcpyHostToDevice));
    A(hipMemcpy(db, bv.data(), sizeof(double) * m, hipMemcpyHostToDevice));
    A(hipMemcpy(dc, cv.data(), sizeof(double) * n, hipMemcpyHostToDevice));
    if (e != hipSuccess) {
        release();
        return BDU_EDEVICE;
    }
    std::vector<const double *> Bs(streams, db), Cs(streams, dc);
    std::vector<int> rs(streams, 1);
    Tuned best{0, 0, 0, 0.0};
    const int k0s[] = {6, 12, 18}, nws[] = {1, 2, 3, 4, 5, 7, 8, 15}, rpls[] = {1, 2};
    int status = BDU_OK;
    for (int k0 : k0s)
        for (int nw : nws)
            for (int rpl : rpls) {
                if (!tiling_supported(k0, nw, rpl)) continue;
                std::vector<bdu_handle> hs(streams, nullptr);
                int s = BDU_OK;
                for (int i = 0; i < streams && s == BDU_OK; ++i)
                    s = create_impl(m, n, dQ, dd, de, dP, k0, nw, rpl, &hs[i]);
                bdu_batch b = nullptr;
                float ms = 0.0f;
                if (s == BDU_OK) s = batch_build(hs.data(), streams, 1, true, &b);
                if (s == BDU_OK) {
                    // one eager step, then three graph steps (the first captures)
                    s = bdu_batch_update(b, Bs.data(), Cs.data(), rs.data());
                    if (s == BDU_OK) s = bdu_batch_update(b, Bs.data(), Cs.data(), rs.data());
                    if (s == BDU_OK) s = bdu_batch_sync(b);
                    if (s == BDU_OK && hipEventRecord(t0, b->stream) != hipSuccess) s = BDU_EDEVICE;
                    for (int k = 0; k < 2 && s == BDU_OK; ++k) s = bdu_batch_update(b, Bs.data(), Cs.data(), rs.data());
                    if (s == BDU_OK && hipEventRecord(t1, b->stream) != hipSuccess) s = BDU_EDEVICE;
                    if (s == BDU_OK) s = bdu_batch_sync(b);
                    if (s == BDU_OK && hipEventElapsedTime(&ms, t0, t1) != hipSuccess) s = BDU_EDEVICE;
                }
                if (b) bdu_batch_destroy(b);
                for (bdu_handle h : hs)
                    if (h) bdu_destroy(h);
                if (s == BDU_ENOMEM) {  // this tiling does not fit: skip it
                    (void)hipGetLastError();
                    continue;
                }
                if (s != BDU_OK) {
                    status = s;
                    break;
                }
                const double us = 1e3 * ms / 2;
                if (best.k0 == 0 || us < best.us) best = Tuned{k0, nw, rpl, us};
            }
    release();
    if (status != BDU_OK) return status;
    if (best.k0 == 0) return BDU_ENOMEM;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_tuned[{m, n}] = best;
    }
    if (out) {
        out[0] = best.k0;
        out[1] = best.nw;
        out[2] = best.rpl;
        out[3] = (int64_t)best.us;
    }
    return BDU_OK;
}

int bdu_tune_save(const char *path)
{
    if (!path) return BDU_EINVAL;
    FILE *f = fopen(path, "w");
    if (!f) return BDU_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    fprintf(f, "# bdu applier tiling per shape: m n k0 nw rows_per_lane us_per_step\n");
    for (auto &kv : g_tuned)
        fprintf(f, "%lld %lld %d %d %d %.1f\n", (long long)kv.first.first, (long long)kv.first.second, kv.second.k0,
                kv.second.nw, kv.second.rpl, kv.second.us);
    return fclose(f) == 0 ? BDU_OK : BDU_EINVAL;
}

int bdu_tune_load(const char *path)
{
    if (!path) return BDU_EINVAL;
    FILE *f = fopen(path, "r");
    if (!f) return BDU_EINVAL;
    char line[256];
    int count = 0;
    std::map<std::pair<int64_t, int64_t>, Tuned> got;
    while (fgets(line, sizeof line, f)) {
        if (line[0] == '#' || line[0] == '\n') continue;
        long long m, n;
        int k0, nw, rpl;
        double us;
        if (sscanf(line, "%lld %lld %d %d %d %lf", &m, &n, &k0, &nw, &rpl, &us) != 6 || m < n || n < 2 ||
            !tiling_supported(k0, nw, rpl)) {
            fclose(f);
            return BDU_EINVAL;
        }
        got[{m, n}] = Tuned{k0, nw, rpl, us};
        ++count;
    }
    fclose(f);
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto &kv : got) g_tuned[kv.first] = kv.second;
    return count;
}

int bdu_timing_enable(int on)
{
    std::lock_guard<std::mutex> lk(g_tmu);
    for (auto &p : g_events) {
        (void)hipEventSynchronize(p.b);
        g_pool.push_back(p.a);
        g_pool.push_back(p.b);
    }
    g_events.clear();
    g_timing = on != 0;
    return BDU_OK;
}

int bdu_timing_read(double *ms, int64_t *launches)
{
    if (!ms || !launches) return BDU_EINVAL;
    std::lock_guard<std::mutex> lk(g_tmu);
    for (int i = 0; i < ST_COUNT; ++i) {
        ms[i] = 0.0;
        launches[i] = 0;
    }
    for (auto &p : g_events) {
        if (hipEventSynchronize(p.b) != hipSuccess) return BDU_EDEVICE;
        float t = 0.f;
        if (hipEventElapsedTime(&t, p.a, p.b) != hipSuccess) return BDU_EDEVICE;
        ms[p.stage] += t;
        launches[p.stage] += 1;
    }
    return BDU_OK;
}

int bdu_givens_device(const double *a, const double *b, int mode, double *c, double *s, double *r, int64_t count)
{
    if (!a || !b || !c || !s || !r || count < 0 || (mode != 1 && mode != 2)) return BDU_EINVAL;
    if (count == 0) return BDU_OK;
    double *buf = nullptr;
    if (hipMalloc(&buf, sizeof(double) * 5 * count) != hipSuccess) return BDU_ENOMEM;
    hipError_t e = hipMemcpy(buf, a, sizeof(double) * count, hipMemcpyDefault);
    if (e == hipSuccess) e = hipMemcpy(buf + count, b, sizeof(double) * count, hipMemcpyDefault);
    if (e == hipSuccess) e = launch_givens(buf, buf + count, mode, buf + 2 * count, buf + 3 * count, buf + 4 * count,
                                           count, nullptr);
    if (e == hipSuccess) e = hipMemcpy(c, buf + 2 * count, sizeof(double) * count, hipMemcpyDefault);
    if (e == hipSuccess) e = hipMemcpy(s, buf + 3 * count, sizeof(double) * count, hipMemcpyDefault);
    if (e == hipSuccess) e = hipMemcpy(r, buf + 4 * count, sizeof(double) * count, hipMemcpyDefault);
    (void)hipFree(buf);
    return e == hipSuccess ? BDU_OK : BDU_EDEVICE;
}

int bdu_plan_stats(int64_t m, int64_t n, int64_t *out)
{
    if (!out || m < n || n < 2) return BDU_EINVAL;
    int k0, nw, rpl;
    tiling_for(m, n, &k0, &nw, &rpl);
    hipError_t e;
    Plan *p = get_plan(m, n, k0, nw, false, &e);
    out[0] = p->nleft + p->nspike;
    out[1] = p->nright;
    out[2] = p->nspike;
    out[3] = (int64_t)p->chains.size();
    out[4] = p->ticks;
    out[5] = p->slots[0];
    out[6] = p->slots[1];
    out[7] = p->L;
    out[8] = p->split;
    return BDU_OK;
}

int bdu_plan_segments(int64_t m, int64_t n, int32_t *tcut, int32_t *bcut, int32_t *block, int64_t cap)
{
    if (m < n || n < 2) return BDU_EINVAL;
    int k0, nw, rpl;
    tiling_for(m, n, &k0, &nw, &rpl);
    hipError_t e;
    Plan *p = get_plan(m, n, k0, nw, false, &e);
    for (int k = 0; k < p->nseg; ++k) {
        if (tcut) tcut[k] = p->tcut[k];
        if (bcut) bcut[k] = p->bcut[k];
    }
    // applier block of each rotation, in the order of bdu_plan_rotations
    int64_t k = 0;
    auto emit = [&](int b) {
        if (block && k < cap) block[k] = b;
        ++k;
    };
    for (int64_t t = 0; t < p->nspike; ++t) emit(-1);
    for (const GenChain &g : p->chains) {
        if (g.type == CH_FOLD) {
            emit(-1);
            continue;
        }
        const int b = chain_in_phase(g.type, g.param) / p->K + (chain_phase(g.type) == 1 ? 0 : p->nb1);
        for (int q = 0; q < g.len; ++q) emit(b);
    }
    return p->nseg;
}

int bdu_plan_blocks(int64_t m, int64_t n, int side, int64_t *out, int64_t cap)
{
    if (m < n || n < 2 || (side != 0 && side != 1) || cap < 0 || (cap > 0 && !out)) return BDU_EINVAL;
    int k0, nw, rpl;
    tiling_for(m, n, &k0, &nw, &rpl);
    hipError_t e;
    Plan *p = get_plan(m, n, k0, nw, false, &e);
    const std::vector<BlockDesc> &bl = p->blocks[side];
    for (size_t b = 0; b < bl.size() && (int64_t)b < cap; ++b) {
        int64_t *o = out + 6 * b;
        o[0] = bl[b].base;
        o[1] = bl[b].lmax;
        o[2] = bl[b].nfront;
        o[3] = bl[b].phase;
        o[4] = bl[b].start;
        o[5] = bl[b].off;
    }
    return (int)bl.size();
}

int64_t bdu_plan_rotations(int64_t m, int64_t n, int32_t *side, int64_t *idx, int32_t *phase, int64_t *tick,
                           int64_t cap)
{
    if (m < n || n < 2) return BDU_EINVAL;
    int k0, nw, rpl;
    tiling_for(m, n, &k0, &nw, &rpl);
    hipError_t e;
    Plan *p = get_plan(m, n, k0, nw, false, &e);
    int64_t k = 0;
    auto emit = [&](int sd, int64_t i, int ph, int64_t tk) {
        if (k < cap) {
            if (side) side[k] = sd;
            if (idx) idx[k] = i;
            if (phase) phase[k] = ph;
            if (tick) tick[k] = tk;
        }
        ++k;
    };
    for (int64_t t = 0; t < p->nspike; ++t) emit(0, m - 1 - t, 0, -1);
    for (const GenChain &g : p->chains) {
        if (g.type == CH_FOLD) {
            emit(2, p->N - 1, 3, g.tau0);
            continue;
        }
        for (int q = 0; q < g.len; ++q) {
            Rot r = decode(g.type, g.param, q);
            emit(r.side, r.i, chain_phase(g.type), (int64_t)g.tau0 + q);
        }
    }
    return k;
}

}  // extern "C"

// ---- orthogonality monitor and correction ----------------------------------------

namespace {

int orth_scratch(bdu_ctx *h)
{
    if (h->orthE) return BDU_OK;
    const int64_t lde = (std::max(h->m, h->n) + 63) / 64 * 64;
    const int64_t ymax = std::max<int64_t>((int64_t)h->hd.ldq * h->m, (int64_t)h->hd.ldp * h->n);
    double *E = nullptr, *Y = nullptr, *part = nullptr, *out = nullptr;
    if (dalloc(h, &E, lde * lde) != hipSuccess || dalloc(h, &Y, ymax) != hipSuccess ||
        dalloc(h, &part, lde) != hipSuccess || dalloc(h, &out, 2) != hipSuccess) {
        (void)hipGetLastError();
        return BDU_ENOMEM;
    }
    h->orthE = E;
    h->orthY = Y;
    h->orthPart = part;
    h->orthOut = out;
    return BDU_OK;
}

// Drift ||X^T X - I||_F of one factor (X: ld x k on the device); with fix,
// one Newton-Schulz step X <- X - X E / 2 when the drift exceeds tol (or
// tol <= 0).
int orth_side(bdu_ctx *h, double *X, int64_t ld, int64_t k, bool fix, double tol, double *err)
{
    const int64_t lde = (k + 63) / 64 * 64;
    hipStream_t st = h->stream;
    double e = 0.0;
    HIPCHK(h, launch_orth_gram(X, ld, k, h->orthE, lde, st));
    HIPCHK(h, launch_orth_norm(h->orthE, k, lde, h->orthPart, h->orthOut, st));
    HIPCHK(h, hipMemcpyAsync(&e, h->orthOut, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(h, hipStreamSynchronize(st));
    if (err) *err = e;
    if (fix && (tol <= 0.0 || e > tol)) {
        HIPCHK(h, launch_orth_update(X, ld, k, h->orthE, lde, h->orthY, st));
        HIPCHK(h, hipMemcpyAsync(X, h->orthY, sizeof(double) * ld * k, hipMemcpyDeviceToDevice, st));
    }
    return BDU_OK;
}

int orth_both(bdu_handle h, bool fix, double tol, double *eq, double *ep)
{
    if (!h) return BDU_EINVAL;
    if (h->poisoned) return BDU_EDEVICE;
    HIPCHK(h, wait_dep(h));
    int st = orth_scratch(h);
    if (st != BDU_OK) return st;
    st = orth_side(h, h->hd.Q, h->hd.ldq, h->m, fix, tol, eq);
    if (st == BDU_OK) st = orth_side(h, h->hd.P, h->hd.ldp, h->n, fix, tol, ep);
    return st;
}

}  // namespace

extern "C" {

int bdu_orth_error(bdu_handle h, double *eq, double *ep)
{
    return orth_both(h, false, 0.0, eq, ep);
}

int bdu_reorthogonalize(bdu_handle h, double tol, double *eq, double *ep)
{
    return orth_both(h, true, tol, eq, ep);
}

}  // extern "C"

// ---- truncated bidiagonal approximation (Section 1.3) ---------------------------

extern "C" int bdu_truncated_bd(bdu_handle h, int64_t r, int64_t *idx, double *err2, double *Qr, double *Pr)
{
    if (!h || r < 1 || r > h->n || r > 65535) return BDU_EINVAL;
    if (h->poisoned) return BDU_EDEVICE;
    HIPCHK(h, wait_dep(h));
    const int64_t m = h->m, n = h->n;
    // per-call scratch, freed before returning
    double *t = nullptr, *er = nullptr, *qr = nullptr, *pr = nullptr;
    int64_t *rank = nullptr, *ix = nullptr;
    hipError_t e = hipMalloc(&t, sizeof(double) * n);
    if (e == hipSuccess) e = hipMalloc(&rank, sizeof(int64_t) * n);
    if (e == hipSuccess) e = hipMalloc(&ix, sizeof(int64_t) * r);
    if (e == hipSuccess) e = hipMalloc(&er, sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&qr, sizeof(double) * m * r);
    if (e == hipSuccess) e = hipMalloc(&pr, sizeof(double) * n * r);
    int st = BDU_OK;
    if (e != hipSuccess) {
        (void)hipGetLastError();
        st = e == hipErrorOutOfMemory ? BDU_ENOMEM : BDU_EDEVICE;
    } else {
        hipStream_t s = h->stream;
        e = launch_trbd(h->hd.Q, h->hd.ldq, m, h->hd.P, h->hd.ldp, n, h->hd.d, h->hd.e, r, t, rank, ix, er, qr, pr,
                        s);
        if (e == hipSuccess && idx) e = copy_out(idx, ix, sizeof(int64_t) * r, s);
        if (e == hipSuccess && err2) e = copy_out(err2, er, sizeof(double), s);
        if (e == hipSuccess && Qr) e = copy_out(Qr, qr, sizeof(double) * m * r, s);
        if (e == hipSuccess && Pr) e = copy_out(Pr, pr, sizeof(double) * n * r, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            h->poisoned = true;
            st = BDU_EDEVICE;
        }
    }
    (void)hipFree(t);
    (void)hipFree(rank);
    (void)hipFree(ix);
    (void)hipFree(er);
    (void)hipFree(qr);
    (void)hipFree(pr);
    return st;
}

// ---- Householder bidiagonal update (Section 3.3, Theorem 1, Algorithm 1) ----------
//
// Column k (then row k) of Q_i^T (B + b c^T) P_j is reached from its factors:
// with S = T^{-1}, Rv = R^{-1} kept explicitly (eq. (TR); a new reflector adds
// the column -S t, t = 2 Y^T y, and a unit diagonal),
//   column: p = e_k - 2 W Rv W^T e_k,  x = B p + b (c^T p),  a = x - 2 Y S^T Y^T x
//   row:    q = e_k - 2 Y S Y^T e_k,   z = B^T q + c (b^T q), a* = z - 2 W Rv^T W^T z
// (the same matrix the representation of Theorem 1 holds; only products with
// the stored reflectors, B, b and c).  B stays the old bidiagonal throughout;
// the new one is written back at the end, with Q <- Q (I - 2 Y S Y^T) and
// P <- P (I - 2 W Rv W^T) (eq. (QP)) on the matrix cores.

namespace {

// One whole update on st (the update vectors are in bst, cst).
hipError_t bhu_record(bdu_ctx *h, hipStream_t st)
{
    const int64_t m = h->m, n = h->n, ldq = h->hd.ldq, ldp = h->hd.ldp;
    double *Y = h->bhu, *Wm = Y + ldq * n, *S = Wm + ldp * n, *Rv = S + ldp * n, *Z1 = Rv + ldp * n,
           *Z2 = Z1 + ldq * n;
    double *vs = Z2 + ldq * n, *vp = vs + ldq, *vx = vp + ldq, *vg = vx + ldq, *vh = vg + ldq, *va = vh + ldq,
           *vt = va + ldq, *vv = vt + ldq, *vq = vv + ldq, *vz = vq + ldq;
    double *dot = vz + ldq, *dp = dot + 64, *ep = dp + ldp, *part = ep + ldp;
    hipError_t a = hipSuccess;
    auto A = [&](hipError_t x) {
        if (a == hipSuccess) a = x;
    };
    // b <- Q^T b, c <- P^T c (into u, v)
    A(launch_project(h->d_self, 1, tiles_of(h), Gate{nullptr, 0, 0}, st));
    A(launch_bhu_copy(Y, nullptr, (ldq + 3 * ldp) * n, st));
    const double *bb = h->hd.u, *cc = h->hd.v, *d = h->hd.d, *e = h->hd.e;
    const int64_t kl = m == n ? n - 1 : n, kr = n - 2;
    // column k of the matrix after i left and j right reflectors, into out
    auto column = [&](int64_t k, int64_t i, int64_t j, double *out) {
        A(launch_bhu_gemv_n(Rv, ldp, j, j, Wm + k, ldp, 1.0, nullptr, -1, vs, part, ldq, st));
        A(launch_bhu_gemv_n(Wm, ldp, n, j, vs, 1, -2.0, nullptr, k, vp, part, ldq, st));
        A(launch_bhu_gemv_t(cc, n, n, 1, vp, 1.0, dot, st));
        A(launch_bhu_bmul(d, e, m, n, vp, bb, dot, vx, st));
        A(launch_bhu_gemv_t(Y, ldq, m, i, vx, 1.0, vg, st));
        A(launch_bhu_gemv_t(S, ldp, i, i, vg, 1.0, vh, st));
        A(launch_bhu_gemv_n(Y, ldq, m, i, vh, 1, -2.0, vx, -1, out, part, ldq, st));
    };
    for (int64_t k = 0; k < kl && a == hipSuccess; ++k) {
        const int64_t j = std::min(k, kr);
        column(k, k, j, va);
        A(launch_bhu_house(va, k, m, dp + k, Y + k * ldq, st));
        A(launch_bhu_gemv_t(Y, ldq, m, k, Y + k * ldq, 2.0, vt, st));
        A(launch_bhu_gemv_n(S, ldp, k + 1, k, vt, 1, -1.0, nullptr, k, S + k * ldp, part, ldq, st));
        if (k >= kr) continue;
        // row k after k + 1 left and j right reflectors
        A(launch_bhu_gemv_n(S, ldp, k + 1, k + 1, Y + k, ldq, 1.0, nullptr, -1, vv, part, ldq, st));
        A(launch_bhu_gemv_n(Y, ldq, m, k + 1, vv, 1, -2.0, nullptr, k, vq, part, ldq, st));
        A(launch_bhu_gemv_t(bb, m, m, 1, vq, 1.0, dot, st));
        A(launch_bhu_btmul(d, e, n, vq, cc, dot, vz, st));
        A(launch_bhu_gemv_t(Wm, ldp, n, j, vz, 1.0, vg, st));
        A(launch_bhu_gemv_t(Rv, ldp, j, j, vg, 1.0, vh, st));
        A(launch_bhu_gemv_n(Wm, ldp, n, j, vh, 1, -2.0, vz, -1, va, part, ldq, st));
        A(launch_bhu_house(va, k + 1, n, ep + k, Wm + k * ldp, st));
        A(launch_bhu_gemv_t(Wm, ldp, n, k, Wm + k * ldp, 2.0, vt, st));
        A(launch_bhu_gemv_n(Rv, ldp, k + 1, k, vt, 1, -1.0, nullptr, k, Rv + k * ldp, part, ldq, st));
    }
    // e_{n-1} (and d_n when m = n) from column n of the final matrix
    column(n - 1, kl, kr, va);
    A(launch_bhu_copy(ep + n - 2, va + n - 2, 1, st));
    if (m == n) A(launch_bhu_copy(dp + n - 1, va + n - 1, 1, st));
    if (kl > 0) {
        A(launch_bhu_gemm(h->hd.Q, ldq, Y, ldq, false, Z1, ldq, m, kl, m, 1.0, 0.0, st));
        A(launch_bhu_gemm(Z1, ldq, S, ldp, false, Z2, ldq, m, kl, kl, 1.0, 0.0, st));
        A(launch_bhu_gemm(Z2, ldq, Y, ldq, true, h->hd.Q, ldq, m, m, kl, -2.0, 1.0, st));
    }
    if (kr > 0) {
        A(launch_bhu_gemm(h->hd.P, ldp, Wm, ldp, false, Z1, ldq, n, kr, n, 1.0, 0.0, st));
        A(launch_bhu_gemm(Z1, ldq, Rv, ldp, false, Z2, ldq, n, kr, kr, 1.0, 0.0, st));
        A(launch_bhu_gemm(Z2, ldq, Wm, ldp, true, h->hd.P, ldp, n, n, kr, -2.0, 1.0, st));
    }
    A(launch_bhu_copy(h->hd.d, dp, n, st));
    A(launch_bhu_copy(h->hd.e, ep, n - 1, st));
    return a;
}

}  // namespace

extern "C" int bdu_update_householder(bdu_handle h, const double *b, const double *c)
{
    if (!h || !b || !c) return BDU_EINVAL;
    if (h->poisoned) return BDU_EDEVICE;
    HIPCHK(h, wait_dep(h));
    const int64_t m = h->m, n = h->n, ldq = h->hd.ldq, ldp = h->hd.ldp;
    if (!h->bhu) {
        const int64_t total = n * (3 * ldq + 3 * ldp) + 10 * ldq + 64 + 2 * ldp + (n + 127) / 128 * ldq;
        if (dalloc(h, &h->bhu, total) != hipSuccess) {
            (void)hipGetLastError();
            return BDU_ENOMEM;
        }
    }
    hipStream_t st = h->stream;
    HIPCHK(h, copy_in(h->hd.bst, b, sizeof(double) * m, st));
    HIPCHK(h, copy_in(h->hd.cst, c, sizeof(double) * n, st));
    const int fin = check_finite(h, {{h->hd.bst, m}, {h->hd.cst, n}}, st);
    if (fin != BDU_OK) return fin;
    // About 80 000 dependent launches at n = 2048; replaying them from a
    // recorded graph measured no faster (the chain of dependent kernels on
    // the device, not the host's launch rate, sets the time).
    HIPCHK(h, bhu_record(h, st));
    return BDU_OK;
}

// ---- subspace tracking (Section 4) ---------------------------------------------

struct bdu_track_ctx {
    int64_t m = 0, n = 0, r = 0;
    // middle factorizations: [0] (r+1) x (r+1) (both sides augmented),
    // [1] (r+1) x r (one side augmented), [2] r x r (neither); [1] and [2]
    // are created on first use.  All run on the stream of [0].
    bdu_handle mid[3] = {nullptr, nullptr, nullptr};
    double *U[2] = {nullptr, nullptr}, *V[2] = {nullptr, nullptr};
    int cur = 0;                   // U[cur], V[cur] hold the tracked factors
    double *d = nullptr, *e = nullptr;
    double *b = nullptr, *c = nullptr;    // staged update vectors
    double *bh = nullptr, *ch = nullptr;  // projections (r)
    double *sh = nullptr;                 // second-pass projections (2 r)
    double *bp = nullptr, *cp = nullptr;  // complements, then unit vectors
    double *mu = nullptr, *mv = nullptr;  // the middle pass's inputs (r + 1)
    double *part = nullptr;               // chunk partials of the projections
    double *npart = nullptr;              // chunk partials of the squared norms
    double *sums = nullptr;               // squared norms, two passes (8, device)
    int *kdrop = nullptr;                 // removed index (device)
    double *h_sums = nullptr;             // pinned: the squared norms
    int *h_k = nullptr;                   // pinned: removed index
    double last_norm[2] = {0.0, 0.0};     // delta, gamma of the last update
    bool have_last = false;
    // drift monitor of U and V (scratch allocated on first use): X padded
    // to ld rows, its Newton-Schulz image, E = X^T X - I, the norm's partials
    double *oX = nullptr, *oY = nullptr, *oE = nullptr, *oPart = nullptr, *oOut = nullptr;
    int64_t oLd = 0, oLde = 0;
    int64_t check_period = 0, since_check = 0, checks = 0, corrections = 0;
    double check_tol = 0.0, drift[2] = {0.0, 0.0};
    bool poisoned = false;
    std::vector<void *> allocs;
    std::vector<void *> pinned;
};

namespace {

template <typename T>
hipError_t talloc(bdu_track_ctx *t, T **p, int64_t count)
{
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, (size_t)std::max<int64_t>(count, 1) * sizeof(T));
    if (e == hipSuccess) {
        t->allocs.push_back(q);
        *p = (T *)q;
    }
    return e;
}

void track_free(bdu_track_ctx *t)
{
    if (t->mid[0]) (void)hipStreamSynchronize(t->mid[0]->stream);
    for (void *p : t->allocs) (void)hipFree(p);
    for (void *p : t->pinned) (void)hipHostFree(p);
    for (bdu_handle h : t->mid)
        if (h) bdu_destroy(h);
    delete t;
}

TrackSides track_sides(bdu_track_ctx *t)
{
    TrackSides s;
    s.side[0] = TrackSide{t->U[t->cur], t->m, t->r, t->m, t->b, t->bh, t->bp};
    s.side[1] = TrackSide{t->V[t->cur], t->n, t->r, t->n, t->c, t->ch, t->cp};
    return s;
}

// The middle handle of shape rows x cols (Q = P = I, B = 0; reset before
// every pass), created on first use on the tracker's stream.
int track_mid(bdu_track_ctx *t, int which, int64_t rows, int64_t cols)
{
    if (t->mid[which]) return BDU_OK;
    std::vector<double> Iq((size_t)(rows * rows), 0.0), Ip((size_t)(cols * cols), 0.0), z((size_t)rows, 0.0);
    for (int64_t i = 0; i < rows; ++i) Iq[(size_t)(i + i * rows)] = 1.0;
    for (int64_t i = 0; i < cols; ++i) Ip[(size_t)(i + i * cols)] = 1.0;
    bdu_handle h = nullptr;
    int st = bdu_create(rows, cols, Iq.data(), z.data(), z.data(), Ip.data(), &h);
    if (st != BDU_OK) return st;
    if (which != 0) {
        st = bdu_set_stream(h, t->mid[0]->stream);
        if (st != BDU_OK) {
            bdu_destroy(h);
            return st;
        }
    }
    t->mid[which] = h;
    return BDU_OK;
}

// Drift ||X^T X - I||_F of the tracked U and V (Section 4.2: the products
// of the thin factors with the middle factors lose orthogonality slowly and
// are reorthogonalized now and then), and with fix one Newton-Schulz step
// X <- X - X E / 2 on each side whose drift exceeds tol (every side if
// tol <= 0).  The orthogonality kernels take X with a leading dimension that
// is a multiple of 128 and zero rows past the matrix, so each side is staged
// in a padded copy.  Synchronizes the tracker's stream.
int track_orth(bdu_track_ctx *t, bool fix, double tol, double *out)
{
    hipStream_t s = t->mid[0]->stream;
    const int64_t r = t->r;
    if (!t->oX) {
        const int64_t ld = (std::max(t->m, t->n) + 127) / 128 * 128, lde = (r + 63) / 64 * 64;
        hipError_t e = talloc(t, &t->oX, ld * r);
        if (e == hipSuccess) e = talloc(t, &t->oY, ld * r);
        if (e == hipSuccess) e = talloc(t, &t->oE, lde * lde);
        if (e == hipSuccess) e = talloc(t, &t->oPart, lde);
        if (e == hipSuccess) e = talloc(t, &t->oOut, 2);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            t->oX = nullptr;  // the pieces already taken are freed with the tracker
            return e == hipErrorOutOfMemory ? BDU_ENOMEM : BDU_EDEVICE;
        }
        t->oLd = ld;
        t->oLde = lde;
    }
    const int64_t ld = t->oLd, lde = t->oLde;
    const size_t row = sizeof(double);
    for (int k = 0; k < 2; ++k) {
        double *X = k == 0 ? t->U[t->cur] : t->V[t->cur];
        const int64_t rows = k == 0 ? t->m : t->n;
        double e = 0.0;
        if (hipMemsetAsync(t->oX, 0, row * ld * r, s) != hipSuccess ||
            hipMemcpy2DAsync(t->oX, row * ld, X, row * rows, row * rows, r, hipMemcpyDeviceToDevice, s) !=
                hipSuccess ||
            launch_orth_gram(t->oX, ld, r, t->oE, lde, s) != hipSuccess ||
            launch_orth_norm(t->oE, r, lde, t->oPart, t->oOut, s) != hipSuccess ||
            hipMemcpyAsync(&e, t->oOut, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            t->poisoned = true;
            return BDU_EDEVICE;
        }
        out[k] = e;
        if (fix && (tol <= 0.0 || e > tol)) {
            if (launch_orth_update(t->oX, ld, r, t->oE, lde, t->oY, s) != hipSuccess ||
                hipMemcpy2DAsync(X, row * rows, t->oY, row * ld, row * rows, r, hipMemcpyDeviceToDevice, s) !=
                    hipSuccess) {
                t->poisoned = true;
                return BDU_EDEVICE;
            }
            ++t->corrections;
        }
    }
    return BDU_OK;
}

}  // namespace

extern "C" {

int bdu_track_create(int64_t m, int64_t n, int64_t r, const double *U, const double *d, const double *e,
                     const double *V, bdu_track *out)
{
    if (!out || !U || !d || !V || (r > 1 && !e) || r < 1 || m < r || n < r || r + 1 > 65535 ||
        m > (int64_t)1 << 30 || n > (int64_t)1 << 30)
        return BDU_EINVAL;
    *out = nullptr;
    const int64_t R = r + 1;
    bdu_track_ctx *t = new bdu_track_ctx;
    t->m = m;
    t->n = n;
    t->r = r;
    int st = track_mid(t, 0, R, R);
    if (st != BDU_OK) {
        track_free(t);
        return st;
    }
    hipError_t e2 = hipSuccess;
    auto A = [&](hipError_t x) {
        if (e2 == hipSuccess) e2 = x;
    };
    for (int k = 0; k < 2; ++k) {
        A(talloc(t, &t->U[k], m * r));
        A(talloc(t, &t->V[k], n * r));
    }
    A(talloc(t, &t->d, r));
    A(talloc(t, &t->e, r));
    A(talloc(t, &t->b, m));
    A(talloc(t, &t->c, n));
    A(talloc(t, &t->bh, R));
    A(talloc(t, &t->ch, R));
    A(talloc(t, &t->sh, 2 * r));
    A(talloc(t, &t->bp, m));
    A(talloc(t, &t->cp, n));
    A(talloc(t, &t->mu, R));
    A(talloc(t, &t->mv, R));
    const int64_t nchunk = (std::max(m, n) + kTrackChunk - 1) / kTrackChunk;
    A(talloc(t, &t->part, 2 * nchunk * r));
    A(talloc(t, &t->npart, 4 * nchunk));
    A(talloc(t, &t->sums, 8));
    A(talloc(t, &t->kdrop, 1));
    if (e2 == hipSuccess) {
        A(hipHostMalloc((void **)&t->h_sums, 8 * sizeof(double), hipHostMallocDefault));
        if (e2 == hipSuccess) t->pinned.push_back(t->h_sums);
        A(hipHostMalloc((void **)&t->h_k, sizeof(int), hipHostMallocDefault));
        if (e2 == hipSuccess) t->pinned.push_back(t->h_k);
    }
    if (e2 != hipSuccess) {
        track_free(t);
        (void)hipGetLastError();
        return e2 == hipErrorOutOfMemory ? BDU_ENOMEM : BDU_EDEVICE;
    }
    hipStream_t s = t->mid[0]->stream;
    A(copy_in(t->U[0], U, sizeof(double) * m * r, s));
    A(copy_in(t->V[0], V, sizeof(double) * n * r, s));
    A(copy_in(t->d, d, sizeof(double) * r, s));
    if (r > 1) A(copy_in(t->e, e, sizeof(double) * (r - 1), s));
    A(hipStreamSynchronize(s));
    if (e2 != hipSuccess) {
        track_free(t);
        return BDU_EDEVICE;
    }
    st = check_finite(t->mid[0], {{t->U[0], m * r}, {t->V[0], n * r}, {t->d, r}, {t->e, r - 1}}, s);
    if (st != BDU_OK) {
        track_free(t);
        return st;
    }
    *out = t;
    return BDU_OK;
}

int bdu_track_update(bdu_track t, const double *b, const double *c)
{
    if (!t || !b || !c) return BDU_EINVAL;
    if (t->poisoned) return BDU_EDEVICE;
    for (bdu_handle h : t->mid)
        if (h && h->poisoned) return BDU_EDEVICE;
    bdu_ctx *m0 = t->mid[0];
    hipStream_t s = m0->stream;
#define TCHK(expr)                        \
    do {                                  \
        if ((expr) != hipSuccess) {       \
            t->poisoned = true;           \
            return BDU_EDEVICE;           \
        }                                 \
    } while (0)
    for (bdu_handle h : t->mid)
        if (h) TCHK(wait_dep(h));
    TCHK(copy_in(t->b, b, sizeof(double) * t->m, s));
    TCHK(copy_in(t->c, c, sizeof(double) * t->n, s));
    int st = check_finite(m0, {{t->b, t->m}, {t->c, t->n}}, s);
    if (st != BDU_OK) return st;
    const TrackSides sides = track_sides(t);
    const int64_t rows = std::max(t->m, t->n), r = t->r;
    // eq. (defup): projections, complements and their squared norms
    TCHK(launch_track_project(sides, rows, r, t->part, s));
    TCHK(launch_track_complement(sides, rows, t->npart, t->sums, s));
    TCHK(hipMemcpyAsync(t->h_sums, t->sums, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
    TCHK(hipStreamSynchronize(s));
    // a second pass for each side whose first complement kept less than
    // half of the squared norm ("twice is enough", Kahan and Parlett)
    double sum2[2] = {-1.0, -1.0};
    int mask = 0;
    for (int k = 0; k < 2; ++k)
        if (!(2.0 * t->h_sums[2 * k + 1] >= t->h_sums[2 * k])) mask |= 1 << k;
    if (mask) {
        TrackSides again = sides;
        for (int k = 0; k < 2; ++k) {
            TrackSide &x = again.side[k];
            x.x = x.xperp;  // project the complement, subtract in place
            x.xhat = t->sh + k * r;
            if (!((mask >> k) & 1)) x.rows = 0;  // this side keeps its first pass
        }
        TCHK(launch_track_project(again, rows, r, t->part, s));
        TCHK(launch_track_complement(again, rows, t->npart, t->sums + 4, s));
        TCHK(launch_track_accumulate(sides, t->sh, r, mask, s));
        TCHK(hipMemcpyAsync(t->h_sums + 4, t->sums + 4, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
        TCHK(hipStreamSynchronize(s));
        for (int k = 0; k < 2; ++k)
            if ((mask >> k) & 1) sum2[k] = t->h_sums[4 + 2 * k + 1];
    }
    // a complement no larger than the worst-case rounding error of the
    // projection sums, rows * 2^-53 * ||x||, carries no direction
    double nrm[2];
    for (int k = 0; k < 2; ++k) {
        const double s0 = t->h_sums[2 * k], s1 = t->h_sums[2 * k + 1];
        const double tau = (double)(k == 0 ? t->m : t->n) * 0x1p-53;
        const double floor2 = tau * tau * s0;
        if (2.0 * s1 >= s0)
            nrm[k] = s1 > floor2 ? std::sqrt(s1) : 0.0;
        else
            nrm[k] = (sum2[k] > floor2 && 2.0 * sum2[k] >= s1) ? std::sqrt(sum2[k]) : 0.0;
    }
    const bool ab = nrm[0] > 0.0, ac = nrm[1] > 0.0;
    if ((!ab || !ac) && r < 2) return BDU_ESPAN;  // no pass on a 2 x 1 or 1 x 1 matrix
    // eq. (qrlr): the appended unit columns
    TCHK(launch_track_scale(sides, rows, nrm[0], nrm[1], s));
    // eq. (equivlrup): one BGU pass on the middle matrix (the r x (r+1) one
    // as its reversed transpose)
    const int which = (ab && ac) ? 0 : ((ab || ac) ? 1 : 2);
    const int64_t pm = which == 2 ? r : r + 1, pn = which == 0 ? r + 1 : r;
    st = track_mid(t, which, pm, pn);
    if (st != BDU_OK) return st;
    bdu_ctx *mh = t->mid[which];
    TrackMiddle mid{mh->hd.Q, mh->hd.P, mh->hd.d, mh->hd.e, mh->hd.ldq, mh->hd.ldp, (int)pm, (int)pn,
                    {ab ? 1 : 0, ac ? 1 : 0}, (!ab && ac) ? 1 : 0};
    TCHK(launch_track_setup(mid, sides, t->d, t->e, r, nrm[0], nrm[1], t->mu, t->mv, s));
    st = bdu_update_projected(mh, t->mu, t->mv);
    if (st != BDU_OK) {
        t->poisoned = true;
        return st;
    }
    // truncation and eq. (bdlrup)
    const int nxt = 1 - t->cur;
    TCHK(launch_track_finish(sides, mid, t->d, t->e, t->kdrop, rows, r, t->U[nxt], t->V[nxt], s));
    TCHK(hipMemcpyAsync(t->h_k, t->kdrop, sizeof(int), hipMemcpyDeviceToHost, s));
    t->cur = nxt;
    t->last_norm[0] = nrm[0];
    t->last_norm[1] = nrm[1];
    t->have_last = true;
#undef TCHK
    if (t->check_period > 0 && ++t->since_check >= t->check_period) {
        t->since_check = 0;
        ++t->checks;
        return track_orth(t, true, t->check_tol, t->drift);
    }
    return BDU_OK;
}

int bdu_track_sync(bdu_track t)
{
    if (!t) return BDU_EINVAL;
    if (t->poisoned) return BDU_EDEVICE;
    return hipStreamSynchronize(t->mid[0]->stream) == hipSuccess ? BDU_OK : BDU_EDEVICE;
}

int bdu_track_read(bdu_track t, double *U, double *d, double *e, double *V)
{
    if (!t) return BDU_EINVAL;
    if (t->poisoned) return BDU_EDEVICE;
    hipStream_t s = t->mid[0]->stream;
    if (hipStreamSynchronize(s) != hipSuccess) return BDU_EDEVICE;
    if (U && copy_out(U, t->U[t->cur], sizeof(double) * t->m * t->r, s) != hipSuccess) return BDU_EDEVICE;
    if (V && copy_out(V, t->V[t->cur], sizeof(double) * t->n * t->r, s) != hipSuccess) return BDU_EDEVICE;
    if (d && copy_out(d, t->d, sizeof(double) * t->r, s) != hipSuccess) return BDU_EDEVICE;
    if (e && t->r > 1 && copy_out(e, t->e, sizeof(double) * (t->r - 1), s) != hipSuccess) return BDU_EDEVICE;
    return hipStreamSynchronize(s) == hipSuccess ? BDU_OK : BDU_EDEVICE;
}

int bdu_track_last(bdu_track t, double *delta, double *gamma, int64_t *dropped)
{
    if (!t) return BDU_EINVAL;
    if (t->poisoned) return BDU_EDEVICE;
    if (!t->have_last) return BDU_EINVAL;
    if (hipStreamSynchronize(t->mid[0]->stream) != hipSuccess) return BDU_EDEVICE;
    if (delta) *delta = t->last_norm[0];
    if (gamma) *gamma = t->last_norm[1];
    if (dropped) *dropped = *t->h_k;
    return BDU_OK;
}

int bdu_track_last_projection(bdu_track t, double *bh, double *ch, double *qb, double *qc)
{
    if (!t) return BDU_EINVAL;
    if (t->poisoned) return BDU_EDEVICE;
    if (!t->have_last) return BDU_EINVAL;
    hipStream_t s = t->mid[0]->stream;
    if (hipStreamSynchronize(s) != hipSuccess) return BDU_EDEVICE;
    if (bh && copy_out(bh, t->bh, sizeof(double) * t->r, s) != hipSuccess) return BDU_EDEVICE;
    if (ch && copy_out(ch, t->ch, sizeof(double) * t->r, s) != hipSuccess) return BDU_EDEVICE;
    if (qb && copy_out(qb, t->bp, sizeof(double) * t->m, s) != hipSuccess) return BDU_EDEVICE;
    if (qc && copy_out(qc, t->cp, sizeof(double) * t->n, s) != hipSuccess) return BDU_EDEVICE;
    return hipStreamSynchronize(s) == hipSuccess ? BDU_OK : BDU_EDEVICE;
}

int bdu_track_orth_error(bdu_track t, double *eu, double *ev)
{
    if (!t) return BDU_EINVAL;
    if (t->poisoned) return BDU_EDEVICE;
    double out[2];
    const int st = track_orth(t, false, 0.0, out);
    if (st != BDU_OK) return st;
    if (eu) *eu = out[0];
    if (ev) *ev = out[1];
    return BDU_OK;
}

int bdu_track_reorthogonalize(bdu_track t, double tol, double *eu, double *ev)
{
    if (!t || !(tol == tol)) return BDU_EINVAL;
    if (t->poisoned) return BDU_EDEVICE;
    double out[2];
    const int st = track_orth(t, true, tol, out);
    if (st != BDU_OK) return st;
    if (eu) *eu = out[0];
    if (ev) *ev = out[1];
    return BDU_OK;
}

int bdu_track_set_drift_check(bdu_track t, int64_t period, double tol)
{
    if (!t || period < 0 || !(tol == tol)) return BDU_EINVAL;
    t->check_period = period;
    t->check_tol = tol;
    t->since_check = 0;
    return BDU_OK;
}

int bdu_track_drift_stats(bdu_track t, int64_t *checks, int64_t *corrections, double *eu, double *ev)
{
    if (!t) return BDU_EINVAL;
    if (checks) *checks = t->checks;
    if (corrections) *corrections = t->corrections;
    if (eu) *eu = t->drift[0];
    if (ev) *ev = t->drift[1];
    return BDU_OK;
}

int bdu_track_destroy(bdu_track t)
{
    if (!t) return BDU_EINVAL;
    track_free(t);
    return BDU_OK;
}

}  // extern "C"
