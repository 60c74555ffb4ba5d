// serve_core.h -- the host side of the served form of the update: resident
// streams grouped in size classes, admission by a device-memory budget,
// bounded per-stream FIFO queues and continuous batching in rounds.  No
// device code: the device work goes through a Backend (serve.cpp binds it
// to the library's handles and batches; a host-only backend drives the same
// logic on the CPU under the sanitizers).
//
// A rank-r request is r rank-1 passes (Section 3.2, eq. (rk1)).  Each size
// class has its own worker and round pipeline: a round takes, from every
// stream of the class with pending work (up to max_batch, oldest request
// first), the next pass of the stream's oldest request and runs them as one
// batched rank-1 step.  A stream's passes thus run in submission order and
// each result is the one the stream would get alone; a rank-1 request
// finishes in one round of its class whatever the ranks of the others, and
// small streams never wait for a round of large ones.
#pragma once
#include <stddef.h>
#include <stdint.h>

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

namespace bdu_serve {

// Status codes are the library's; the core passes the backend's through and
// uses these itself.
constexpr int kOk = BDU_OK, kEinval = BDU_EINVAL, kEnomem = BDU_ENOMEM, kEbusy = BDU_EBUSY;

struct Backend {
    virtual ~Backend() = default;
    // Device bytes a resident m x n stream takes (negative: a status).
    virtual int64_t footprint(int64_t m, int64_t n) = 0;
    // Make a resident factorization for size class cls.
    virtual int open(int cls, int64_t m, int64_t n, const double *Q, const double *d, const double *e,
                     const double *P, void **h) = 0;
    virtual int close(void *h) = 0;
    virtual int read(void *h, double *Q, double *d, double *e, double *P) = 0;
    // Copy bytes from a host or device pointer into host memory.
    virtual int fetch(void *dst, const void *src, size_t bytes) = 0;
    // One round of class cls over its current members (the membership is
    // the same while gen is): member k takes one rank-1 pass with Bs[k],
    // Cs[k] when ranks[k] = 1 and nothing when ranks[k] = 0.  Returns when
    // the round's work is complete.
    virtual int round(int cls, uint64_t gen, const std::vector<void *> &members, const double *const *Bs,
                      const double *const *Cs, const int *ranks) = 0;
    // Drop what the backend keeps for class cls's membership (called before a
    // member is closed, with no round of the class running).
    virtual void retire(int cls) = 0;
};

class Core {
public:
    // bounds: ascending upper limits of n for the size classes (a stream goes
    // to the first class whose bound is at least its n, else to one more
    // class after the last); empty: one class.
    Core(Backend *be, int64_t budget, int queue_cap, int max_batch, const std::vector<int64_t> &bounds);
    ~Core();
    int open(int64_t m, int64_t n, const double *Q, const double *d, const double *e, const double *P, int *sid);
    int submit(int sid, const double *B, const double *C, int r, int64_t *ticket);
    int wait(int64_t ticket, double *latency_ms);
    int poll(int64_t ticket);
    int drain();
    int pause(bool paused);
    int read(int sid, double *Q, double *d, double *e, double *P);
    int close(int sid);
    // counts[9]: completed, rejected busy, rejected memory, rounds, batched
    // passes, streams, bytes in use, pending requests, failed; latency[4]:
    // p50, p99, mean, max of completed requests (ms).
    int stats(int64_t *counts, double *latency);
    // Zero the counters and the latency record (streams and queues stay).
    int reset_stats();
    int classes() const { return (int)cls_.size(); }
    int class_of(int64_t n) const;

private:
    using Clock = std::chrono::steady_clock;
    struct Request {
        int64_t ticket = 0;
        int sid = 0, r = 0, next = 0;
        std::vector<double> B, C;  // host copies, m x r and n x r
        Clock::time_point submitted, finished;
        bool done = false, detached = false;
        int status = kOk;
    };
    struct Stream {
        void *h = nullptr;
        int64_t m = 0, n = 0, bytes = 0;
        int cls = 0;
        std::deque<Request *> queue;
        bool in_flight = false;  // its oldest request is in a running round
        bool held = false;       // a read or close is using the handle
        bool closing = false;    // removed from its class: takes no more requests
    };
    struct Class {
        std::vector<int> members;  // stream ids, in the backend's member order
        uint64_t gen = 1;          // bumped on every membership change
        std::mutex round_mu;       // held for a round, and by read/close around the handle
        std::thread worker;
    };

    bool class_has_work(int c) const;
    void run(int c);
    int hold(int sid, Stream **out);

    Backend *be_;
    int64_t budget_, used_ = 0;
    int queue_cap_, max_batch_;
    std::vector<int64_t> bounds_;
    std::vector<std::unique_ptr<Class>> cls_;
    std::mutex copy_mu_;
    mutable std::mutex mu_;
    std::condition_variable cv_work_, cv_done_;
    std::map<int, Stream> streams_;
    int next_sid_ = 1;
    std::unordered_map<int64_t, std::unique_ptr<Request>> reqs_;
    int64_t next_ticket_ = 1;
    bool stop_ = false, paused_ = false;
    int64_t completed_ = 0, rej_busy_ = 0, rej_mem_ = 0, rounds_ = 0, batched_ = 0, failed_ = 0;
    std::vector<double> lat_ms_;
};

}  // namespace bdu_serve
