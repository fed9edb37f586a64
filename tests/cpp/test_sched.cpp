// Host-only tests of the request scheduler (sched.h) with a mock executor: the
// allocator against a granule-bitmap model, FIFO admission under slot and
// memory limits, quantum slicing, deadlines, cancellation and percentiles.
#include "../../paper_2606_12579_amd/csrc/sched.h"

#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <vector>

using namespace gm::sched;

static int failures = 0;
#define CHECK(c)                                                             \
    do {                                                                     \
        if (!(c)) {                                                          \
            std::printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #c);         \
            ++failures;                                                      \
        }                                                                    \
    } while (0)

// first-fit reference on a bitmap of granules
struct Model {
    std::vector<char> used;
    explicit Model(size_t granules) : used(granules, 0) {}
    long first_fit(size_t g) const
    {
        size_t run = 0;
        for (size_t i = 0; i < used.size(); ++i) {
            run = used[i] ? 0 : run + 1;
            if (run == g) return (long)(i + 1 - g);
        }
        return -1;
    }
};

static void test_allocator()
{
    const size_t G = 512;
    Allocator a(G * kGranule + 100);          // the tail below one granule is unusable
    CHECK(a.size() == G * kGranule);
    Model m(G);
    std::mt19937 rng(7);
    std::vector<std::pair<size_t, size_t>> live;
    for (int it = 0; it < 20000; ++it) {
        if (live.empty() || rng() % 3 != 0) {
            const size_t bytes = 1 + rng() % (40 * kGranule);
            const size_t g = (bytes + kGranule - 1) / kGranule;
            size_t off = 0;
            const bool ok = a.alloc(bytes, off);
            const long want = m.first_fit(g);
            CHECK(ok == (want >= 0));
            if (ok) {
                CHECK((long)(off / kGranule) == want);
                CHECK(off % kGranule == 0);
                for (size_t i = 0; i < g; ++i) m.used[off / kGranule + i] = 1;
                live.push_back({off, bytes});
            }
        } else {
            const size_t k = rng() % live.size();
            a.release(live[k].first, live[k].second);
            const size_t g = (live[k].second + kGranule - 1) / kGranule;
            for (size_t i = 0; i < g; ++i) m.used[live[k].first / kGranule + i] = 0;
            live.erase(live.begin() + k);
        }
        size_t used = 0;
        for (char c : m.used) used += c;
        CHECK(a.used() == used * kGranule);
    }
    for (auto &l : live) a.release(l.first, l.second);
    CHECK(a.used() == 0 && a.blocks() == 1 && a.largest() == a.size());
}

struct Mock {
    Req r;
    std::vector<std::pair<int, int>> ranges;
};

static void test_admission_and_slicing()
{
    // budget of 12 granules, 3 slots, quantum 7
    Core c(12 * kGranule, 3, 7, 100);
    std::vector<Mock> q(8);
    const size_t sizes[8] = {4, 4, 4, 3, 9, 1, 1, 2};
    const int steps[8] = {10, 20, 7, 1, 30, 15, 3, 8};
    double t = 0;
    for (int i = 0; i < 8; ++i) {
        q[i].r.id = i + 1;
        q[i].r.bytes = sizes[i] * kGranule;
        q[i].r.n_steps = steps[i];
        q[i].r.work = steps[i];
        q[i].r.user = &q[i];
        CHECK(c.submit(&q[i].r, t) == 0);
    }
    Req big;
    big.bytes = 13 * kGranule;
    CHECK(c.submit(&big, t) == -1);            // can never fit
    std::vector<Req *> fin;
    std::vector<int> order;
    int cycles = 0;
    while (!c.idle() && cycles < 1000) {
        auto in = c.admit(t, fin);
        for (Req *r : in) order.push_back((int)r->id);
        CHECK(c.active() <= 3);
        CHECK(c.memory().used() <= 12 * kGranule);
        auto plan = c.plan();
        for (auto &s : plan) {
            CHECK(s.k_end - s.k_begin <= 7 && s.k_end > s.k_begin);
            static_cast<Mock *>(s.r->user)->ranges.push_back({s.k_begin, s.k_end});
        }
        c.complete(plan, t, t + 1, fin);
        t += 1;
        ++cycles;
    }
    CHECK(c.idle());
    // FIFO admission order
    for (size_t i = 0; i < order.size(); ++i) CHECK(order[i] == (int)i + 1);
    CHECK(order.size() == 8);
    // each horizon covered exactly once, contiguously, in quanta
    for (auto &m : q) {
        int k = 1;
        for (auto &rg : m.ranges) {
            CHECK(rg.first == k);
            k = rg.second;
        }
        CHECK(k == m.r.n_steps + 1);
        CHECK(m.r.status == 0 && m.r.state == kDone);
    }
    CHECK(fin.size() == 8);
    const Stats s = c.stats();
    CHECK(s.completed == 8 && s.rejected == 1 && s.max_active_seen == 3);
    CHECK(c.memory().used() == 0);
}

static void test_head_of_line_and_joining()
{
    // strict FIFO: a large head waits for memory, the smaller request behind it waits too
    Core c(8 * kGranule, 8, 5, 100);
    Req a, b, d;
    a.id = 1; a.bytes = 6 * kGranule; a.n_steps = 10;
    b.id = 2; b.bytes = 6 * kGranule; b.n_steps = 5;
    d.id = 3; d.bytes = 1 * kGranule; d.n_steps = 5;
    std::vector<Req *> fin;
    c.submit(&a, 0);
    c.admit(0, fin);
    c.submit(&b, 0.5);
    c.submit(&d, 0.6);
    auto in = c.admit(1, fin);
    CHECK(in.empty());                         // b does not fit, d waits behind it
    c.complete(c.plan(), 1, 2, fin);           // a: steps 1..5
    CHECK(c.admit(2, fin).empty());
    c.complete(c.plan(), 2, 3, fin);           // a: 6..10, done
    CHECK(fin.size() == 1 && fin[0] == &a);
    in = c.admit(3, fin);                      // both join now
    CHECK(in.size() == 2 && in[0] == &b && in[1] == &d);
    CHECK(b.t_admit == 3 && b.t_admit - b.t_submit == 2.5);
}

static void test_deadlines_and_cancel()
{
    Core c(100 * kGranule, 1, 10, 100);
    Req a, b, d, e;
    a.id = 1; a.bytes = kGranule; a.n_steps = 100; a.deadline = 2.5;   // expires while active
    b.id = 2; b.bytes = kGranule; b.n_steps = 5; b.deadline = 1.0;     // expires while waiting
    d.id = 3; d.bytes = kGranule; d.n_steps = 5;                        // cancelled while waiting
    e.id = 4; e.bytes = kGranule; e.n_steps = 5;
    std::vector<Req *> fin;
    for (Req *r : {&a, &b, &d, &e}) c.submit(r, 0);
    c.admit(0, fin);
    CHECK(c.cancel(3));
    CHECK(!c.cancel(99));
    double t = 0;
    while (!c.idle() && t < 100) {
        c.admit(t, fin);
        c.complete(c.plan(), t, t + 1, fin);
        t += 1;
    }
    CHECK(a.status == -5 && b.status == -5 && d.status == -6 && e.status == 0);
    CHECK(a.t_admit == 0 && b.t_admit < 0 && d.t_admit < 0);
    const Stats s = c.stats();
    CHECK(s.expired == 2 && s.cancelled == 1 && s.completed == 1);
    CHECK(c.memory().used() == 0);
}

// a request cancelled while the cycle that covers its whole horizon runs is
// reported cancelled, not completed (its work on the device may have stopped)
static void test_cancel_during_last_cycle()
{
    Core c(100 * kGranule, 4, 10, 100);
    Req a;
    a.id = 1; a.bytes = kGranule; a.n_steps = 10;
    std::vector<Req *> fin;
    c.submit(&a, 0);
    c.admit(0, fin);
    const std::vector<Slice> run = c.plan();
    CHECK(run.size() == 1 && run[0].k_begin == 1 && run[0].k_end == 11);
    CHECK(c.cancel(1));                        // raised while the cycle runs
    c.complete(run, 0, 1, fin);
    CHECK(fin.size() == 1 && a.status == -6);
    const Stats s = c.stats();
    CHECK(s.cancelled == 1 && s.completed == 0);
    CHECK(c.memory().used() == 0);
}

static void test_queue_limit_and_percentiles()
{
    Core c(1000 * kGranule, 1000, 1000, 3);
    Req r[5];
    std::vector<Req *> fin;
    for (int i = 0; i < 5; ++i) {
        r[i].id = i + 1;
        r[i].bytes = kGranule;
        r[i].n_steps = 1;
    }
    for (int i = 0; i < 3; ++i) CHECK(c.submit(&r[i], 0.1 * i) == 0);
    CHECK(c.submit(&r[3], 0.3) == -4);         // queue full
    c.admit(1, fin);
    c.complete(c.plan(), 1, 2.0, fin);         // finish at t = 2: latencies 2.0, 1.9, 1.8
    const Stats s = c.stats();
    // linear interpolation between order statistics (1.8, 1.9, 2.0)
    CHECK(std::abs(s.p50_s - 1.9) < 1e-12);
    CHECK(std::abs(s.p99_s - (1.9 + 0.98 * 0.1)) < 1e-12);
    CHECK(std::abs(s.max_s - 2.0) < 1e-12 && std::abs(s.mean_s - 1.9) < 1e-12);
}

int main()
{
    test_allocator();
    test_admission_and_slicing();
    test_head_of_line_and_joining();
    test_deadlines_and_cancel();
    test_cancel_during_last_cycle();
    test_queue_limit_and_percentiles();
    if (failures) {
        std::printf("%d failures\n", failures);
        return 1;
    }
    std::printf("sched OK\n");
    return 0;
}
