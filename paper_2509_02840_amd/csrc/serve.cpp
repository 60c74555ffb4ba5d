// serve.cpp -- the served form of the update: resident streams, admission by
// a device-memory budget, bounded per-stream queues and continuous batching.
//
// One worker thread owns the GPU work.  A rank-r request is r rank-1 passes
// (Section 3.2, eq. (rk1)), and rounds batch passes, not requests: each round takes,
// from every stream with pending work (up to max_batch streams, oldest
// request first), the next pass of the stream's oldest request and runs them
// together as one batched rank-1 update (bdu_update_batched).  A stream's
// passes thus run in submission order and each result is the one its stream
// would get alone; a rank-1 request finishes in one round whatever the ranks
// of the others, and requests that arrive during a round join the next.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/bdu.h"

namespace {

using Clock = std::chrono::steady_clock;

double ms_since(Clock::time_point t0, Clock::time_point t1)
{
    return std::chrono::duration<double, std::milli>(t1 - t0).count();
}

struct Request {
    int64_t ticket;
    int sid;
    int r;
    std::vector<double> B, C;  // host copies, m x r and n x r
    Clock::time_point submitted, finished;
    int next = 0;  // next column (pass) to run
    bool done = false;
    bool detached = false;  // no ticket was handed out: released when done
    int status = BDU_OK;
};

struct Stream {
    bdu_handle h = nullptr;
    int64_t m = 0, n = 0, bytes = 0;
    std::deque<Request *> queue;
    bool in_flight = false;  // its oldest request is in the running round
    bool held = false;       // a read or close is using the handle
};

bool on_device(const void *p)
{
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice;
}

// Copy `bytes` from a host or device pointer into host memory.  Device
// sources go through a non-blocking stream of their own, so a submission
// never waits for a running round.
int fetch(void *dst, const void *src, size_t bytes, hipStream_t copy_stream)
{
    if (!on_device(src)) {
        memcpy(dst, src, bytes);
        return BDU_OK;
    }
    if (hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, copy_stream) != hipSuccess ||
        hipStreamSynchronize(copy_stream) != hipSuccess)
        return BDU_EDEVICE;
    return BDU_OK;
}

}  // namespace

struct bdu_server_ctx {
    int64_t budget = 0, used = 0;
    int queue_cap = 1, max_batch = 1;
    hipStream_t stream = nullptr;       // the rounds
    hipStream_t copy_stream = nullptr;  // submissions from device memory
    std::mutex copy_mu;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::map<int, Stream> streams;
    int next_sid = 1;
    std::unordered_map<int64_t, std::unique_ptr<Request>> reqs;
    int64_t next_ticket = 1;
    bool stop = false, paused = false;
    std::thread worker;
    // statistics
    int64_t completed = 0, rej_busy = 0, rej_mem = 0, rounds = 0, batched = 0, failed = 0;
    std::vector<double> lat_ms;

    bool has_work() const
    {
        for (auto &kv : streams)
            if (!kv.second.queue.empty() && !kv.second.held) return true;
        return false;
    }

    void run();
};

void bdu_server_ctx::run()
{
    std::vector<Request *> round;
    std::vector<bdu_handle> hs;
    std::vector<const double *> Bs, Cs;
    std::vector<int> rs;
    for (;;) {
        round.clear();
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait(lk, [&] { return stop || (!paused && has_work()); });
            if (stop && !has_work()) return;
            if (stop && paused) return;
            // the streams' oldest requests, oldest first
            std::vector<std::pair<Clock::time_point, int>> ready;
            for (auto &kv : streams)
                if (!kv.second.queue.empty() && !kv.second.held)
                    ready.push_back({kv.second.queue.front()->submitted, kv.first});
            std::sort(ready.begin(), ready.end());
            if ((int)ready.size() > max_batch) ready.resize(max_batch);
            hs.clear();
            Bs.clear();
            Cs.clear();
            rs.clear();
            for (auto &x : ready) {
                Stream &s = streams[x.second];
                s.in_flight = true;
                Request *q = s.queue.front();
                round.push_back(q);
                hs.push_back(s.h);
                Bs.push_back(q->B.data() + (size_t)q->next * s.m);
                Cs.push_back(q->C.data() + (size_t)q->next * s.n);
                rs.push_back(1);
            }
        }
        const int st = bdu_update_batched(hs.data(), Bs.data(), Cs.data(), rs.data(), (int)round.size());
        const Clock::time_point t = Clock::now();
        {
            std::lock_guard<std::mutex> lk(mu);
            ++rounds;
            batched += (int64_t)round.size();
            for (Request *q : round) {
                Stream &s = streams[q->sid];
                s.in_flight = false;
                if (st == BDU_OK && ++q->next < q->r) continue;  // more passes to run
                s.queue.pop_front();
                q->finished = t;
                q->status = st;
                q->done = true;
                if (st == BDU_OK) {
                    ++completed;
                    lat_ms.push_back(ms_since(q->submitted, t));
                } else {
                    ++failed;
                }
                q->B.clear();
                q->B.shrink_to_fit();
                q->C.clear();
                q->C.shrink_to_fit();
                if (q->detached) reqs.erase(q->ticket);
            }
        }
        cv_done.notify_all();
    }
}

extern "C" {

int bdu_server_create(int64_t budget_bytes, int queue_cap, int max_batch, bdu_server *out)
{
    if (!out || budget_bytes <= 0 || queue_cap < 1 || max_batch < 1) return BDU_EINVAL;
    auto s = std::make_unique<bdu_server_ctx>();
    s->budget = budget_bytes;
    s->queue_cap = queue_cap;
    s->max_batch = max_batch;
    // non-blocking: neither waits for work the client issues on the null stream
    if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) return BDU_EDEVICE;
    if (hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipStreamDestroy(s->stream);
        return BDU_EDEVICE;
    }
    bdu_server_ctx *p = s.get();
    s->worker = std::thread([p] { p->run(); });
    *out = s.release();
    return BDU_OK;
}

int bdu_server_open(bdu_server s, int64_t m, int64_t n, const double *Q, const double *d, const double *e,
                    const double *P, int *stream_id)
{
    if (!s || !stream_id || m < n || n < 2 || !Q || !d || !e || !P) return BDU_EINVAL;
    const int64_t need = bdu_footprint_bytes(m, n);
    if (need < 0) return (int)need;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->used + need > s->budget) {
            ++s->rej_mem;
            return BDU_ENOMEM;
        }
        s->used += need;  // reserved while the handle is created
    }
    bdu_handle h = nullptr;
    int st = bdu_create(m, n, Q, d, e, P, &h);
    if (st == BDU_OK) st = bdu_set_stream(h, s->stream);
    std::lock_guard<std::mutex> lk(s->mu);
    if (st != BDU_OK) {
        if (h) bdu_destroy(h);
        s->used -= need;
        if (st == BDU_ENOMEM) ++s->rej_mem;
        return st;
    }
    const int sid = s->next_sid++;
    Stream &x = s->streams[sid];
    x.h = h;
    x.m = m;
    x.n = n;
    x.bytes = need;
    *stream_id = sid;
    return BDU_OK;
}

int bdu_server_submit(bdu_server s, int stream_id, const double *B, const double *C, int r, int64_t *ticket)
{
    if (!s || !B || !C || r < 1) return BDU_EINVAL;
    int64_t m, n;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->streams.find(stream_id);
        if (it == s->streams.end()) return BDU_EINVAL;
        if ((int)it->second.queue.size() >= s->queue_cap) {
            ++s->rej_busy;
            return BDU_EBUSY;
        }
        m = it->second.m;
        n = it->second.n;
    }
    auto q = std::make_unique<Request>();
    q->sid = stream_id;
    q->r = r;
    q->B.resize((size_t)(m * r));
    q->C.resize((size_t)(n * r));
    int st;
    {
        std::lock_guard<std::mutex> lk(s->copy_mu);
        st = fetch(q->B.data(), B, sizeof(double) * m * r, s->copy_stream);
        if (st == BDU_OK) st = fetch(q->C.data(), C, sizeof(double) * n * r, s->copy_stream);
    }
    if (st != BDU_OK) return st;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->streams.find(stream_id);
        if (it == s->streams.end()) return BDU_EINVAL;
        if ((int)it->second.queue.size() >= s->queue_cap) {
            ++s->rej_busy;
            return BDU_EBUSY;
        }
        q->submitted = Clock::now();
        q->ticket = s->next_ticket++;
        q->detached = ticket == nullptr;
        if (ticket) *ticket = q->ticket;
        it->second.queue.push_back(q.get());
        s->reqs[q->ticket] = std::move(q);
    }
    s->cv_work.notify_one();
    return BDU_OK;
}

int bdu_server_wait(bdu_server s, int64_t ticket, double *latency_ms)
{
    if (!s) return BDU_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return BDU_EINVAL;
    Request *q = it->second.get();
    s->cv_done.wait(lk, [&] { return q->done; });
    if (latency_ms) *latency_ms = ms_since(q->submitted, q->finished);
    const int st = q->status;
    s->reqs.erase(it);
    return st;
}

int bdu_server_poll(bdu_server s, int64_t ticket)
{
    if (!s) return BDU_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return BDU_EINVAL;
    return it->second->done ? 1 : 0;
}

int bdu_server_drain(bdu_server s)
{
    if (!s) return BDU_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->paused) return BDU_EINVAL;  // would never finish
    s->cv_done.wait(lk, [&] {
        for (auto &kv : s->streams)
            if (!kv.second.queue.empty()) return false;
        return true;
    });
    return BDU_OK;
}

int bdu_server_pause(bdu_server s, int paused)
{
    if (!s) return BDU_EINVAL;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->paused = paused != 0;
    }
    s->cv_work.notify_all();
    return BDU_OK;
}

// Hold a stream's handle: wait until none of its requests is queued or
// running, and keep the worker off it until released.
static int hold(bdu_server s, int stream_id, Stream **out)
{
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->streams.find(stream_id);
    if (it == s->streams.end() || it->second.held) return BDU_EINVAL;
    if (s->paused && !it->second.queue.empty()) return BDU_EINVAL;  // would never drain
    Stream &x = it->second;
    s->cv_done.wait(lk, [&] { return x.queue.empty() && !x.in_flight; });
    x.held = true;
    *out = &x;
    return BDU_OK;
}

int bdu_server_read(bdu_server s, int stream_id, double *Q, double *d, double *e, double *P)
{
    if (!s) return BDU_EINVAL;
    Stream *x = nullptr;
    int st = hold(s, stream_id, &x);
    if (st != BDU_OK) return st;
    st = bdu_read(x->h, Q, d, e, P);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        x->held = false;
    }
    s->cv_work.notify_one();
    return st;
}

int bdu_server_close(bdu_server s, int stream_id)
{
    if (!s) return BDU_EINVAL;
    Stream *x = nullptr;
    int st = hold(s, stream_id, &x);
    if (st != BDU_OK) return st;
    st = bdu_destroy(x->h);
    std::lock_guard<std::mutex> lk(s->mu);
    s->used -= x->bytes;
    s->streams.erase(stream_id);
    return st;
}

int bdu_server_stats(bdu_server s, int64_t *counts, double *latency)
{
    if (!s) return BDU_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    if (counts) {
        int64_t pending = 0;
        for (auto &kv : s->streams) pending += (int64_t)kv.second.queue.size();
        counts[0] = s->completed;
        counts[1] = s->rej_busy;
        counts[2] = s->rej_mem;
        counts[3] = s->rounds;
        counts[4] = s->batched;
        counts[5] = (int64_t)s->streams.size();
        counts[6] = s->used;
        counts[7] = pending;
        counts[8] = s->failed;
    }
    if (latency) {
        std::vector<double> v = s->lat_ms;
        std::sort(v.begin(), v.end());
        auto pct = [&](double p) {
            if (v.empty()) return 0.0;
            size_t k = (size_t)std::min<double>(v.size() - 1, std::max(0.0, p * (double)(v.size() - 1) + 0.5));
            return v[k];
        };
        double sum = 0;
        for (double x : v) sum += x;
        latency[0] = pct(0.50);
        latency[1] = pct(0.99);
        latency[2] = v.empty() ? 0.0 : sum / (double)v.size();
        latency[3] = v.empty() ? 0.0 : v.back();
    }
    return BDU_OK;
}

int bdu_server_destroy(bdu_server s)
{
    if (!s) return BDU_EINVAL;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    for (auto &kv : s->streams) bdu_destroy(kv.second.h);
    // requests never run (destroyed while paused) are reported failed
    {
        std::lock_guard<std::mutex> lk(s->mu);
        for (auto &kv : s->reqs)
            if (!kv.second->done) {
                kv.second->done = true;
                kv.second->status = BDU_EINVAL;
            }
    }
    s->cv_done.notify_all();
    if (s->stream) (void)hipStreamDestroy(s->stream);
    if (s->copy_stream) (void)hipStreamDestroy(s->copy_stream);
    delete s;
    return BDU_OK;
}

}  // extern "C"
