// serve.cpp -- the served form's C ABI (bdu_server_*) over the host core of
// serve_core.h, with the device work on the library's handles and batches.
//
// Each size class keeps one persistent batch (bdu_batch_*) over all of its
// resident streams, rebuilt only when the class's membership changes; a
// round is one step of that batch with rank 1 for the streams it serves and
// rank 0 for the others, so rounds allocate nothing.  The streams of a class
// share one HIP stream; every class has its own, so the classes' rounds run
// concurrently on the device.  The batches launch eagerly: their steps are
// queued by the workers while clients use the device from other threads,
// which a stream capture must not overlap.
#include <hip/hip_runtime.h>
#include <string.h>

#include <memory>
#include <vector>

#include "../../include/bdu.h"
#include "serve_core.h"

namespace {

bool on_device(const void *p)
{
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice;
}

class HipBackend : public bdu_serve::Backend {
public:
    struct PerClass {
        hipStream_t stream = nullptr;
        bdu_batch batch = nullptr;  // touched only under the class's round lock
        uint64_t gen = 0;
    };

    int init(int classes)
    {
        cls_.resize((size_t)classes);
        // non-blocking: none waits for work the client issues on the null stream
        if (hipStreamCreateWithFlags(&copy_stream_, hipStreamNonBlocking) != hipSuccess) return BDU_EDEVICE;
        for (auto &k : cls_)
            if (hipStreamCreateWithFlags(&k.stream, hipStreamNonBlocking) != hipSuccess) return BDU_EDEVICE;
        return BDU_OK;
    }

    ~HipBackend() override
    {
        for (auto &k : cls_) {
            if (k.batch) bdu_batch_destroy(k.batch);
            if (k.stream) (void)hipStreamDestroy(k.stream);
        }
        if (copy_stream_) (void)hipStreamDestroy(copy_stream_);
    }

    int64_t footprint(int64_t m, int64_t n) override { return bdu_footprint_bytes(m, n); }

    int open(int cls, int64_t m, int64_t n, const double *Q, const double *d, const double *e, const double *P,
             void **out) override
    {
        bdu_handle h = nullptr;
        int st = bdu_create(m, n, Q, d, e, P, &h);
        if (st == BDU_OK) st = bdu_set_stream(h, cls_[(size_t)cls].stream);
        if (st != BDU_OK) {
            if (h) bdu_destroy(h);
            return st;
        }
        *out = h;
        return BDU_OK;
    }

    int close(void *h) override { return bdu_destroy((bdu_handle)h); }

    int read(void *h, double *Q, double *d, double *e, double *P) override
    {
        return bdu_read((bdu_handle)h, Q, d, e, P);
    }

    // Device sources go through a stream of their own, so a submission
    // never waits for a running round.
    int fetch(void *dst, const void *src, size_t bytes) override
    {
        if (!on_device(src)) {
            memcpy(dst, src, bytes);
            return BDU_OK;
        }
        if (hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, copy_stream_) != hipSuccess ||
            hipStreamSynchronize(copy_stream_) != hipSuccess)
            return BDU_EDEVICE;
        return BDU_OK;
    }

    int round(int cls, uint64_t gen, const std::vector<void *> &members, const double *const *Bs,
              const double *const *Cs, const int *ranks) override
    {
        PerClass &k = cls_[(size_t)cls];
        if (!k.batch || k.gen != gen) {
            retire(cls);
            std::vector<bdu_handle> hs(members.size());
            for (size_t i = 0; i < members.size(); ++i) hs[i] = (bdu_handle)members[i];
            const int st = bdu_batch_create_flags(hs.data(), (int)hs.size(), 1, BDU_BATCH_EAGER, &k.batch);
            if (st != BDU_OK) {
                k.batch = nullptr;
                return st;
            }
            k.gen = gen;
        }
        int st = bdu_batch_update(k.batch, Bs, Cs, ranks);
        if (st == BDU_OK) st = bdu_batch_sync(k.batch);
        if (st != BDU_OK) retire(cls);
        return st;
    }

    void retire(int cls) override
    {
        PerClass &k = cls_[(size_t)cls];
        if (k.batch) bdu_batch_destroy(k.batch);
        k.batch = nullptr;
    }

private:
    std::vector<PerClass> cls_;
    hipStream_t copy_stream_ = nullptr;
};

}  // namespace

// The backend is declared first so that it outlives the core (whose
// destructor stops the workers and closes the streams through it).
struct bdu_server_ctx {
    HipBackend backend;
    std::unique_ptr<bdu_serve::Core> core;
};

extern "C" {

int bdu_server_create_classes(int64_t budget_bytes, int queue_cap, int max_batch, const int64_t *bounds,
                              int nbounds, bdu_server *out)
{
    if (!out || budget_bytes <= 0 || queue_cap < 1 || max_batch < 1 || nbounds < 0 || nbounds > 15 ||
        (nbounds > 0 && !bounds))
        return BDU_EINVAL;
    *out = nullptr;
    std::vector<int64_t> b(bounds, bounds + nbounds);
    for (int i = 0; i < nbounds; ++i)
        if (b[(size_t)i] < 2 || (i > 0 && b[(size_t)i] <= b[(size_t)i - 1])) return BDU_EINVAL;
    auto s = std::make_unique<bdu_server_ctx>();
    const int st = s->backend.init(nbounds + 1);
    if (st != BDU_OK) return st;
    s->core = std::make_unique<bdu_serve::Core>(&s->backend, budget_bytes, queue_cap, max_batch, b);
    *out = s.release();
    return BDU_OK;
}

int bdu_server_create(int64_t budget_bytes, int queue_cap, int max_batch, bdu_server *out)
{
    static const int64_t kBounds[] = {1024, 2048, 4096};
    return bdu_server_create_classes(budget_bytes, queue_cap, max_batch, kBounds, 3, out);
}

int bdu_server_open(bdu_server s, int64_t m, int64_t n, const double *Q, const double *d, const double *e,
                    const double *P, int *stream_id)
{
    return s ? s->core->open(m, n, Q, d, e, P, stream_id) : BDU_EINVAL;
}

int bdu_server_submit(bdu_server s, int stream_id, const double *B, const double *C, int r, int64_t *ticket)
{
    return s ? s->core->submit(stream_id, B, C, r, ticket) : BDU_EINVAL;
}

int bdu_server_wait(bdu_server s, int64_t ticket, double *latency_ms)
{
    return s ? s->core->wait(ticket, latency_ms) : BDU_EINVAL;
}

int bdu_server_poll(bdu_server s, int64_t ticket)
{
    return s ? s->core->poll(ticket) : BDU_EINVAL;
}

int bdu_server_drain(bdu_server s)
{
    return s ? s->core->drain() : BDU_EINVAL;
}

int bdu_server_pause(bdu_server s, int paused)
{
    return s ? s->core->pause(paused != 0) : BDU_EINVAL;
}

int bdu_server_read(bdu_server s, int stream_id, double *Q, double *d, double *e, double *P)
{
    return s ? s->core->read(stream_id, Q, d, e, P) : BDU_EINVAL;
}

int bdu_server_close(bdu_server s, int stream_id)
{
    return s ? s->core->close(stream_id) : BDU_EINVAL;
}

int bdu_server_stats(bdu_server s, int64_t *counts, double *latency)
{
    return s ? s->core->stats(counts, latency) : BDU_EINVAL;
}

int bdu_server_reset_stats(bdu_server s)
{
    return s ? s->core->reset_stats() : BDU_EINVAL;
}

int bdu_server_class_of(bdu_server s, int64_t n)
{
    return s ? s->core->class_of(n) : BDU_EINVAL;
}

int bdu_server_destroy(bdu_server s)
{
    if (!s) return BDU_EINVAL;
    s->core.reset();
    delete s;
    return BDU_OK;
}

}  // extern "C"
