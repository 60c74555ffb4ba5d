// serve_core.cpp -- the host side of the served form (serve_core.h).
//
// Locks: a class's round_mu is always taken before mu_, never the other way
// round.  A worker holds its class's round_mu for a whole round (selection,
// the backend's device work, and nothing else of the core), so read and
// close, which take it around their use of a handle, never overlap a round
// of the handle's class, and a membership change is only seen by the next
// round.
#include "serve_core.h"

#include <string.h>

#include <algorithm>

namespace bdu_serve {

namespace {

double ms_between(std::chrono::steady_clock::time_point t0, std::chrono::steady_clock::time_point t1)
{
    return std::chrono::duration<double, std::milli>(t1 - t0).count();
}

}  // namespace

Core::Core(Backend *be, int64_t budget, int queue_cap, int max_batch, const std::vector<int64_t> &bounds)
    : be_(be), budget_(budget), queue_cap_(queue_cap), max_batch_(max_batch), bounds_(bounds)
{
    for (size_t c = 0; c <= bounds_.size(); ++c) cls_.push_back(std::make_unique<Class>());
    for (int c = 0; c < (int)cls_.size(); ++c) cls_[c]->worker = std::thread([this, c] { run(c); });
}

Core::~Core()
{
    {
        std::lock_guard<std::mutex> lk(mu_);
        stop_ = true;
    }
    cv_work_.notify_all();
    for (auto &k : cls_)
        if (k->worker.joinable()) k->worker.join();
    for (int c = 0; c < (int)cls_.size(); ++c) be_->retire(c);
    for (auto &kv : streams_) be_->close(kv.second.h);
    {
        // requests never run (destroyed while paused) are reported failed
        std::lock_guard<std::mutex> lk(mu_);
        for (auto &kv : reqs_)
            if (!kv.second->done) {
                kv.second->done = true;
                kv.second->status = kEinval;
            }
    }
    cv_done_.notify_all();
}

int Core::class_of(int64_t n) const
{
    for (size_t i = 0; i < bounds_.size(); ++i)
        if (n <= bounds_[i]) return (int)i;
    return (int)bounds_.size();
}

bool Core::class_has_work(int c) const
{
    for (int sid : cls_[c]->members) {
        const Stream &s = streams_.at(sid);
        if (!s.queue.empty() && !s.held) return true;
    }
    return false;
}

void Core::run(int c)
{
    Class &k = *cls_[c];
    std::vector<void *> hs;
    std::vector<const double *> Bs, Cs;
    std::vector<int> rs;
    std::vector<Request *> round;
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(mu_);
            cv_work_.wait(lk, [&] { return stop_ || (!paused_ && class_has_work(c)); });
            if (stop_ && (paused_ || !class_has_work(c))) return;
        }
        std::lock_guard<std::mutex> rl(k.round_mu);
        uint64_t gen;
        round.clear();
        {
            std::lock_guard<std::mutex> lk(mu_);
            if (paused_ || !class_has_work(c)) continue;  // changed while the round lock was taken
            gen = k.gen;
            const size_t cnt = k.members.size();
            hs.assign(cnt, nullptr);
            Bs.assign(cnt, nullptr);
            Cs.assign(cnt, nullptr);
            rs.assign(cnt, 0);
            // the class's oldest requests, oldest first
            std::vector<std::pair<Clock::time_point, size_t>> ready;
            for (size_t i = 0; i < cnt; ++i) {
                Stream &s = streams_.at(k.members[i]);
                hs[i] = s.h;
                if (!s.queue.empty() && !s.held) ready.push_back({s.queue.front()->submitted, i});
            }
            std::sort(ready.begin(), ready.end());
            if ((int)ready.size() > max_batch_) ready.resize(max_batch_);
            for (auto &x : ready) {
                Stream &s = streams_.at(k.members[x.second]);
                s.in_flight = true;
                Request *q = s.queue.front();
                round.push_back(q);
                Bs[x.second] = q->B.data() + (size_t)q->next * s.m;
                Cs[x.second] = q->C.data() + (size_t)q->next * s.n;
                rs[x.second] = 1;
            }
        }
        const int st = be_->round(c, gen, hs, Bs.data(), Cs.data(), rs.data());
        const Clock::time_point t = Clock::now();
        {
            std::lock_guard<std::mutex> lk(mu_);
            ++rounds_;
            batched_ += (int64_t)round.size();
            for (Request *q : round) {
                Stream &s = streams_.at(q->sid);
                s.in_flight = false;
                if (st == kOk && ++q->next < q->r) continue;  // more passes to run
                s.queue.pop_front();
                q->finished = t;
                q->status = st;
                q->done = true;
                if (st == kOk) {
                    ++completed_;
                    lat_ms_.push_back(ms_between(q->submitted, t));
                } else {
                    ++failed_;
                }
                q->B.clear();
                q->B.shrink_to_fit();
                q->C.clear();
                q->C.shrink_to_fit();
                if (q->detached) reqs_.erase(q->ticket);
            }
        }
        cv_done_.notify_all();
    }
}

int Core::open(int64_t m, int64_t n, const double *Q, const double *d, const double *e, const double *P, int *sid)
{
    if (!sid || m < n || n < 2 || !Q || !d || !e || !P) return kEinval;
    const int64_t need = be_->footprint(m, n);
    if (need < 0) return (int)need;
    const int c = class_of(n);
    {
        std::lock_guard<std::mutex> lk(mu_);
        if (used_ + need > budget_) {
            ++rej_mem_;
            return kEnomem;
        }
        used_ += need;  // reserved while the backend creates the stream
    }
    void *h = nullptr;
    const int st = be_->open(c, m, n, Q, d, e, P, &h);
    std::lock_guard<std::mutex> lk(mu_);
    if (st != kOk) {
        used_ -= need;
        if (st == kEnomem) ++rej_mem_;
        return st;
    }
    const int id = next_sid_++;
    Stream &x = streams_[id];
    x.h = h;
    x.m = m;
    x.n = n;
    x.bytes = need;
    x.cls = c;
    cls_[c]->members.push_back(id);
    ++cls_[c]->gen;
    *sid = id;
    return kOk;
}

int Core::submit(int sid, const double *B, const double *C, int r, int64_t *ticket)
{
    if (!B || !C || r < 1) return kEinval;
    int64_t m, n;
    {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = streams_.find(sid);
        if (it == streams_.end() || it->second.closing) return kEinval;
        if ((int)it->second.queue.size() >= queue_cap_) {
            ++rej_busy_;
            return kEbusy;
        }
        m = it->second.m;
        n = it->second.n;
    }
    auto q = std::make_unique<Request>();
    q->sid = sid;
    q->r = r;
    q->B.resize((size_t)(m * r));
    q->C.resize((size_t)(n * r));
    int st;
    {
        std::lock_guard<std::mutex> lk(copy_mu_);
        st = be_->fetch(q->B.data(), B, sizeof(double) * (size_t)(m * r));
        if (st == kOk) st = be_->fetch(q->C.data(), C, sizeof(double) * (size_t)(n * r));
    }
    if (st != kOk) return st;
    {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = streams_.find(sid);
        if (it == streams_.end() || it->second.closing) return kEinval;
        if ((int)it->second.queue.size() >= queue_cap_) {
            ++rej_busy_;
            return kEbusy;
        }
        q->submitted = Clock::now();
        q->ticket = next_ticket_++;
        q->detached = ticket == nullptr;
        if (ticket) *ticket = q->ticket;
        it->second.queue.push_back(q.get());
        reqs_[q->ticket] = std::move(q);
    }
    cv_work_.notify_all();  // the workers of every class wait on it
    return kOk;
}

int Core::wait(int64_t ticket, double *latency_ms)
{
    std::unique_lock<std::mutex> lk(mu_);
    auto it = reqs_.find(ticket);
    if (it == reqs_.end()) return kEinval;
    Request *q = it->second.get();
    cv_done_.wait(lk, [&] { return q->done; });
    if (latency_ms) *latency_ms = ms_between(q->submitted, q->finished);
    const int st = q->status;
    reqs_.erase(it);
    return st;
}

int Core::poll(int64_t ticket)
{
    std::lock_guard<std::mutex> lk(mu_);
    auto it = reqs_.find(ticket);
    if (it == reqs_.end()) return kEinval;
    return it->second->done ? 1 : 0;
}

int Core::drain()
{
    std::unique_lock<std::mutex> lk(mu_);
    if (paused_) return kEinval;  // would never finish
    cv_done_.wait(lk, [&] {
        for (auto &kv : streams_)
            if (!kv.second.queue.empty()) return false;
        return true;
    });
    return kOk;
}

int Core::pause(bool paused)
{
    {
        std::lock_guard<std::mutex> lk(mu_);
        paused_ = paused;
    }
    cv_work_.notify_all();
    return kOk;
}

// Hold a stream's handle: wait until none of its requests is queued or
// running, and keep rounds and submissions off it until released.
int Core::hold(int sid, Stream **out)
{
    std::unique_lock<std::mutex> lk(mu_);
    auto it = streams_.find(sid);
    if (it == streams_.end() || it->second.held) return kEinval;
    if (paused_ && !it->second.queue.empty()) return kEinval;  // would never drain
    Stream &x = it->second;
    cv_done_.wait(lk, [&] { return x.queue.empty() && !x.in_flight; });
    x.held = true;
    *out = &x;
    return kOk;
}

int Core::read(int sid, double *Q, double *d, double *e, double *P)
{
    Stream *x = nullptr;
    int st = hold(sid, &x);
    if (st != kOk) return st;
    {
        std::lock_guard<std::mutex> rl(cls_[x->cls]->round_mu);
        st = be_->read(x->h, Q, d, e, P);
    }
    {
        std::lock_guard<std::mutex> lk(mu_);
        x->held = false;
    }
    cv_work_.notify_all();
    return st;
}

int Core::close(int sid)
{
    Stream *x = nullptr;
    int st = hold(sid, &x);
    if (st != kOk) return st;
    Class &k = *cls_[x->cls];
    {
        std::lock_guard<std::mutex> rl(k.round_mu);
        {
            std::lock_guard<std::mutex> lk(mu_);
            k.members.erase(std::find(k.members.begin(), k.members.end(), sid));
            ++k.gen;
            x->closing = true;  // submissions that raced the hold fail
            for (Request *q : x->queue) {
                q->done = true;
                q->status = kEinval;
                q->finished = Clock::now();
                ++failed_;
                if (q->detached) reqs_.erase(q->ticket);
            }
            x->queue.clear();
        }
        cv_done_.notify_all();
        be_->retire(x->cls);
        st = be_->close(x->h);
    }
    std::lock_guard<std::mutex> lk(mu_);
    used_ -= x->bytes;
    streams_.erase(sid);
    return st;
}

int Core::stats(int64_t *counts, double *latency)
{
    std::lock_guard<std::mutex> lk(mu_);
    if (counts) {
        int64_t pending = 0;
        for (auto &kv : streams_) pending += (int64_t)kv.second.queue.size();
        counts[0] = completed_;
        counts[1] = rej_busy_;
        counts[2] = rej_mem_;
        counts[3] = rounds_;
        counts[4] = batched_;
        counts[5] = (int64_t)streams_.size();
        counts[6] = used_;
        counts[7] = pending;
        counts[8] = failed_;
    }
    if (latency) {
        std::vector<double> v = lat_ms_;
        std::sort(v.begin(), v.end());
        auto pct = [&](double p) {
            if (v.empty()) return 0.0;
            const size_t k = (size_t)std::min<double>((double)(v.size() - 1),
                                                      std::max(0.0, p * (double)(v.size() - 1) + 0.5));
            return v[k];
        };
        double sum = 0;
        for (double x : v) sum += x;
        latency[0] = pct(0.50);
        latency[1] = pct(0.99);
        latency[2] = v.empty() ? 0.0 : sum / (double)v.size();
        latency[3] = v.empty() ? 0.0 : v.back();
    }
    return kOk;
}

int Core::reset_stats()
{
    std::lock_guard<std::mutex> lk(mu_);
    completed_ = rej_busy_ = rej_mem_ = rounds_ = batched_ = failed_ = 0;
    lat_ms_.clear();
    return kOk;
}

}  // namespace bdu_serve
