// Drives the served form's host core (serve_core.cpp) with a host-only
// backend under the sanitizers: several client threads submit to streams in
// three size classes, with pauses, queue caps, budget admission, reads and
// closes while other classes run.  Every pass records its update's tag in
// its stream, so the order each stream saw is checked against the order it
// was submitted in.  Exit status 0 when every check holds.
#include <stdio.h>
#include <string.h>

#include <atomic>
#include <chrono>
#include <map>
#include <mutex>
#include <set>
#include <thread>
#include <vector>

#include "../../paper_2509_02840_amd/csrc/serve_core.h"

using bdu_serve::kEbusy;
using bdu_serve::kEinval;
using bdu_serve::kEnomem;
using bdu_serve::kOk;

static std::atomic<int> g_fail{0};
#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c);  \
            ++g_fail;                                                         \
        }                                                                     \
    } while (0)

struct FakeHandle {
    int64_t m, n;
    int cls;
    std::vector<double> log;  // tag of every pass, in order
};

class FakeBackend : public bdu_serve::Backend {
public:
    std::mutex mu;
    std::set<FakeHandle *> alive;
    std::map<int, uint64_t> cached_gen;           // class -> membership the "batch" was built for
    std::map<int, std::vector<void *>> cached;    // class -> that membership
    std::atomic<int64_t> rounds{0};

    int64_t footprint(int64_t m, int64_t n) override { return 8 * (m * m + n * n); }

    int open(int cls, int64_t m, int64_t n, const double *, const double *, const double *, const double *,
             void **h) override
    {
        auto *f = new FakeHandle{m, n, cls, {}};
        std::lock_guard<std::mutex> lk(mu);
        alive.insert(f);
        *h = f;
        return kOk;
    }

    int close(void *h) override
    {
        std::lock_guard<std::mutex> lk(mu);
        CHECK(alive.erase((FakeHandle *)h) == 1);
        for (auto &kv : cached)
            for (void *p : kv.second) CHECK(p != h);  // retired before its handle closes
        delete (FakeHandle *)h;
        return kOk;
    }

    int read(void *h, double *Q, double *d, double *, double *) override
    {
        std::lock_guard<std::mutex> lk(mu);
        auto *f = (FakeHandle *)h;
        CHECK(alive.count(f) == 1);
        d[0] = (double)f->log.size();
        for (size_t i = 0; i < f->log.size() && i < (size_t)(f->m * f->m); ++i) Q[i] = f->log[i];
        return kOk;
    }

    int fetch(void *dst, const void *src, size_t bytes) override
    {
        memcpy(dst, src, bytes);
        return kOk;
    }

    int round(int cls, uint64_t gen, const std::vector<void *> &members, const double *const *Bs,
              const double *const *Cs, const int *ranks) override
    {
        {
            std::lock_guard<std::mutex> lk(mu);
            if (!cached.count(cls) || cached_gen[cls] != gen) {
                cached[cls] = members;
                cached_gen[cls] = gen;
            }
            CHECK(cached[cls] == members);  // same generation, same membership
            for (size_t k = 0; k < members.size(); ++k) {
                auto *f = (FakeHandle *)members[k];
                CHECK(alive.count(f) == 1);
                CHECK(f->cls == cls);
                CHECK(ranks[k] == 0 || ranks[k] == 1);
                if (ranks[k] == 1) {
                    CHECK(Bs[k] && Cs[k]);
                    CHECK(Bs[k][f->m - 1] == -Bs[k][0]);  // the column was copied whole
                    f->log.push_back(Bs[k][0]);
                }
            }
        }
        ++rounds;
        std::this_thread::sleep_for(std::chrono::microseconds(50 + 100 * cls));
        return kOk;
    }

    void retire(int cls) override
    {
        std::lock_guard<std::mutex> lk(mu);
        cached.erase(cls);
        cached_gen.erase(cls);
    }
};

// A request of rank r for a stream of m rows whose passes carry tags
// base, base + 1, ..., in column order.
static std::vector<double> block(int64_t m, int r, double base)
{
    std::vector<double> B((size_t)(m * r), 0.0);
    for (int j = 0; j < r; ++j) {
        B[(size_t)(j * m)] = base + j;
        B[(size_t)(j * m + m - 1)] = -(base + j);
    }
    return B;
}

static void mixed_load()
{
    FakeBackend be;
    {
        bdu_serve::Core core(&be, int64_t(1) << 40, 6, 4, {16, 64});
        CHECK(core.classes() == 3 && core.class_of(16) == 0 && core.class_of(17) == 1 && core.class_of(500) == 2);
        const int64_t shapes[][2] = {{8, 8}, {12, 10}, {40, 40}, {60, 33}, {100, 100}, {130, 90}};
        std::vector<int> sids;
        std::vector<double> z(130 * 130, 0.0);
        for (auto &s : shapes) {
            int sid = 0;
            CHECK(core.open(s[0], s[1], z.data(), z.data(), z.data(), z.data(), &sid) == kOk);
            sids.push_back(sid);
        }
        // client t owns streams t and t + 3; each submits 12 requests per
        // stream with ranks 1..3 and waits for them in a random order
        std::vector<std::vector<double>> expect(sids.size());
        std::mutex emu;
        std::vector<std::thread> clients;
        for (int t = 0; t < 3; ++t)
            clients.emplace_back([&, t] {
                std::vector<int64_t> tickets;
                for (int k = 0; k < 12; ++k)
                    for (int which : {t, t + 3}) {
                        const int64_t m = shapes[which][0], n = shapes[which][1];
                        const int r = 1 + (k + which) % 3;
                        const double base = 1000.0 * (which + 1) + 10.0 * k;
                        auto B = block(m, r, base);
                        std::vector<double> C((size_t)(n * r), 0.5);
                        int64_t tk = 0;
                        int st;
                        while ((st = core.submit(sids[which], B.data(), C.data(), r, &tk)) == kEbusy)
                            std::this_thread::sleep_for(std::chrono::microseconds(200));
                        CHECK(st == kOk);
                        tickets.push_back(tk);
                        std::lock_guard<std::mutex> lk(emu);
                        for (int j = 0; j < r; ++j) expect[which].push_back(base + j);
                    }
                for (size_t i = 0; i < tickets.size(); ++i) {
                    double ms = -1;
                    CHECK(core.wait(tickets[tickets.size() - 1 - i], &ms) == kOk);  // newest first
                    CHECK(ms >= 0);
                }
            });
        // meanwhile: reads of a stream of another class, and a stream opened
        // and closed in the largest class
        std::thread other([&] {
            std::vector<double> Q(130 * 130), d(130), e(130), P(130 * 130);
            for (int k = 0; k < 20; ++k) {
                CHECK(core.read(sids[0], Q.data(), d.data(), e.data(), P.data()) == kOk);
                int sid = 0;
                CHECK(core.open(120, 110, z.data(), z.data(), z.data(), z.data(), &sid) == kOk);
                auto B = block(120, 2, 9.0e6 + k);
                std::vector<double> C(220, 1.0);
                int64_t tk = 0;
                CHECK(core.submit(sid, B.data(), C.data(), 2, &tk) == kOk);
                CHECK(core.wait(tk, nullptr) == kOk);
                CHECK(core.read(sid, Q.data(), d.data(), e.data(), P.data()) == kOk);
                CHECK(d[0] == 2.0 && Q[0] == 9.0e6 + k && Q[1] == 9.0e6 + k + 1);
                CHECK(core.close(sid) == kOk);
            }
        });
        for (auto &c : clients) c.join();
        other.join();
        CHECK(core.drain() == kOk);
        std::vector<double> Q(130 * 130), d(130), e(130), P(130 * 130);
        for (size_t i = 0; i < sids.size(); ++i) {
            CHECK(core.read(sids[i], Q.data(), d.data(), e.data(), P.data()) == kOk);
            CHECK((size_t)d[0] == expect[i].size());
            for (size_t j = 0; j < expect[i].size() && j < (size_t)d[0]; ++j) CHECK(Q[j] == expect[i][j]);
        }
        int64_t c[9];
        double lat[4];
        CHECK(core.stats(c, lat) == kOk);
        CHECK(c[0] == 3 * 2 * 12 + 20 && c[7] == 0 && c[8] == 0 && c[5] == 6);
        CHECK(lat[0] <= lat[1] && lat[1] <= lat[3]);
    }
    CHECK(be.alive.empty());
}

static void admission_and_caps()
{
    FakeBackend be;
    bdu_serve::Core core(&be, 8 * (2 * 32 * 32) * 2 + 100, 2, 8, {});
    std::vector<double> z(64 * 64, 0.0);
    int a = 0, b = 0, c = 0;
    CHECK(core.open(32, 32, z.data(), z.data(), z.data(), z.data(), &a) == kOk);
    CHECK(core.open(32, 32, z.data(), z.data(), z.data(), z.data(), &b) == kOk);
    CHECK(core.open(32, 32, z.data(), z.data(), z.data(), z.data(), &c) == kEnomem);
    CHECK(core.open(4, 8, z.data(), z.data(), z.data(), z.data(), &c) == kEinval);  // m < n
    core.pause(true);
    auto B = block(32, 1, 1.0);
    std::vector<double> C(32, 1.0);
    int64_t t1 = 0, t2 = 0, t3 = 0;
    CHECK(core.submit(a, B.data(), C.data(), 1, &t1) == kOk);
    CHECK(core.submit(a, B.data(), C.data(), 1, &t2) == kOk);
    CHECK(core.submit(a, B.data(), C.data(), 1, &t3) == kEbusy);
    CHECK(core.submit(b, B.data(), C.data(), 1, nullptr) == kOk);  // detached
    CHECK(core.poll(t1) == 0);
    std::vector<double> Q(32 * 32), d(32), e(32), P(32 * 32);
    CHECK(core.read(a, Q.data(), d.data(), e.data(), P.data()) == kEinval);  // paused with work queued
    CHECK(core.drain() == kEinval);
    core.pause(false);
    CHECK(core.wait(t1, nullptr) == kOk && core.wait(t2, nullptr) == kOk);
    CHECK(core.wait(t1, nullptr) == kEinval);  // a ticket is released by its wait
    CHECK(core.drain() == kOk);
    CHECK(core.close(b) == kOk);
    CHECK(core.open(32, 32, z.data(), z.data(), z.data(), z.data(), &c) == kOk && c != b);
    CHECK(core.submit(b, B.data(), C.data(), 1, nullptr) == kEinval);  // closed
    int64_t s[9];
    CHECK(core.stats(s, nullptr) == kOk);
    CHECK(s[0] == 3 && s[1] == 1 && s[2] == 1 && s[5] == 2);
    // destroyed while paused with requests queued: they fail, nothing leaks
    core.pause(true);
    CHECK(core.submit(c, B.data(), C.data(), 1, nullptr) == kOk);
    CHECK(core.submit(a, B.data(), C.data(), 1, &t3) == kOk);
}

int main()
{
    mixed_load();
    admission_and_caps();
    if (g_fail) {
        fprintf(stderr, "%d checks failed\n", g_fail.load());
        return 1;
    }
    printf("serve core: all checks passed\n");
    return 0;
}
