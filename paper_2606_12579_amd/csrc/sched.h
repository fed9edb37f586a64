// Request scheduling of the replanning server, free of any device code so that
// it can be built and tested on its own: a first-fit allocator over the device
// memory budget (memory-based admission), the FIFO of waiting requests, the set
// of active requests (slots), the step quantum each active request advances per
// cycle (continuous batching: requests join and leave between cycles), deadlines,
// cancellation and latency statistics.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <map>
#include <vector>

namespace gm {
namespace sched {

constexpr size_t kGranule = 256;

inline size_t round_up(size_t n) { return (n + kGranule - 1) / kGranule * kGranule; }

// First-fit allocator over [0, size): offsets and lengths in multiples of 256 B.
class Allocator {
public:
    explicit Allocator(size_t size = 0) { reset(size); }
    void reset(size_t size)
    {
        size_ = size / kGranule * kGranule;
        free_.clear();
        if (size_) free_[0] = size_;
        used_ = 0;
    }
    bool alloc(size_t n, size_t &off)
    {
        n = round_up(std::max<size_t>(n, 1));
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                off = it->first;
                const size_t rest = it->second - n;
                free_.erase(it);
                if (rest) free_[off + n] = rest;
                used_ += n;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t n)
    {
        n = round_up(std::max<size_t>(n, 1));
        used_ -= n;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + n == next->first) {   // merge with the following block
            n += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {                            // merge with the preceding block
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += n;
                return;
            }
        }
        free_[off] = n;
    }
    size_t size() const { return size_; }
    size_t used() const { return used_; }
    size_t largest() const
    {
        size_t m = 0;
        for (auto &f : free_) m = std::max(m, f.second);
        return m;
    }
    size_t blocks() const { return free_.size(); }

private:
    size_t size_ = 0, used_ = 0;
    std::map<size_t, size_t> free_;   // offset -> length
};

enum State { kWaiting = 0, kActive = 1, kDone = 2 };

struct Req {
    int64_t id = 0;
    size_t bytes = 0;         // device bytes while active
    size_t off = 0;           // offset in the budget
    int n_steps = 0;          // horizon N_k
    int k_next = 1;           // next step to run
    double work = 0;          // interactions of the whole horizon
    double t_submit = 0, t_admit = -1, t_finish = -1;
    double deadline = 0;      // absolute time, 0 = none
    int status = 0;           // 0 ok, else a negative gmapp_status
    int state = kWaiting;
    bool cancel = false;
    void *user = nullptr;     // executor data
};

struct Stats {
    int64_t submitted = 0, completed = 0, rejected = 0, expired = 0, cancelled = 0, cycles = 0;
    double busy_s = 0;            // time with at least one active request
    double work_done = 0;         // interactions of completed requests
    double p50_s = 0, p99_s = 0, max_s = 0, mean_s = 0;
    double cycle_mean_s = 0;
    int max_active_seen = 0;
    size_t peak_bytes = 0;
};

// One cycle's work for an active request: steps [k_begin, k_end).
struct Slice {
    Req *r;
    int k_begin, k_end;
};

class Core {
public:
    Core(size_t budget, int max_active, int quantum, int max_queue)
        : alloc_(budget), max_active_(max_active), quantum_(quantum), max_queue_(max_queue)
    {
    }

    // Queue a request (ECAPACITY-like -4 when the queue is full, -1 when it can never fit).
    int submit(Req *r, double now)
    {
        ++st_.submitted;
        if (round_up(r->bytes) > alloc_.size()) {
            ++st_.rejected;
            return -1;
        }
        if ((int)wait_.size() >= max_queue_) {
            ++st_.rejected;
            return -4;
        }
        r->t_submit = now;
        r->state = kWaiting;
        wait_.push_back(r);
        return 0;
    }

    // Admit waiting requests in FIFO order while a slot and memory are free;
    // requests past their deadline or cancelled leave the queue as finished.
    std::vector<Req *> admit(double now, std::vector<Req *> &finished)
    {
        std::vector<Req *> in;
        for (auto it = wait_.begin(); it != wait_.end();) {
            Req *r = *it;
            if (r->cancel || (r->deadline > 0 && now > r->deadline)) {
                if (r->status == 0) {
                    r->status = r->cancel ? -6 : -5;
                    (r->cancel ? st_.cancelled : st_.expired)++;
                }
                finish(r, now, finished);
                it = wait_.erase(it);
                continue;
            }
            ++it;
        }
        while (!wait_.empty() && (int)active_.size() < max_active_) {
            Req *r = wait_.front();
            size_t off;
            if (!alloc_.alloc(r->bytes, off)) break;     // strict FIFO: the head waits for memory
            r->off = off;
            r->state = kActive;
            r->t_admit = now;
            wait_.pop_front();
            active_.push_back(r);
            in.push_back(r);
        }
        st_.peak_bytes = std::max(st_.peak_bytes, alloc_.used());
        st_.max_active_seen = std::max(st_.max_active_seen, (int)active_.size());
        return in;
    }

    // The next cycle: every active request advances by the quantum.
    std::vector<Slice> plan() const
    {
        std::vector<Slice> s;
        for (Req *r : active_) s.push_back(Slice{r, r->k_next, std::min(r->k_next + quantum_, r->n_steps + 1)});
        return s;
    }

    // After a cycle ran [t0, t1]: advance the ranges; finished or cancelled
    // requests release their memory and are returned.  A request cancelled while
    // its cycle ran is cancelled even if that cycle reached the end of its horizon:
    // the device may have skipped or stopped its work.
    void complete(const std::vector<Slice> &ran, double t0, double t1, std::vector<Req *> &finished)
    {
        if (!ran.empty()) {
            ++st_.cycles;
            st_.busy_s += t1 - t0;
        }
        for (const Slice &s : ran) s.r->k_next = s.k_end;
        for (auto it = active_.begin(); it != active_.end();) {
            Req *r = *it;
            const bool done = r->k_next > r->n_steps;
            const bool late = !done && r->deadline > 0 && t1 > r->deadline;
            if (done || r->cancel || late) {
                if (r->status == 0 && (r->cancel || !done)) {
                    r->status = r->cancel ? -6 : -5;
                    (r->cancel ? st_.cancelled : st_.expired)++;
                }
                alloc_.release(r->off, r->bytes);
                finish(r, t1, finished);
                it = active_.erase(it);
            } else {
                ++it;
            }
        }
    }

    bool cancel(int64_t id)
    {
        for (Req *r : wait_)
            if (r->id == id) return r->cancel = true;
        for (Req *r : active_)
            if (r->id == id) return r->cancel = true;
        return false;
    }

    bool idle() const { return wait_.empty() && active_.empty(); }
    size_t waiting() const { return wait_.size(); }
    size_t active() const { return active_.size(); }
    const Allocator &memory() const { return alloc_; }
    int quantum() const { return quantum_; }

    Stats stats() const
    {
        Stats s = st_;
        std::vector<double> l = lat_;
        if (!l.empty()) {
            std::sort(l.begin(), l.end());
            auto pct = [&](double q) {             // linear interpolation between order statistics
                const double x = q * (l.size() - 1);
                const size_t i = (size_t)std::floor(x);
                const size_t j = std::min(i + 1, l.size() - 1);
                return l[i] + (x - i) * (l[j] - l[i]);
            };
            s.p50_s = pct(0.50);
            s.p99_s = pct(0.99);
            s.max_s = l.back();
            double sum = 0;
            for (double v : l) sum += v;
            s.mean_s = sum / l.size();
        }
        s.cycle_mean_s = s.cycles ? s.busy_s / s.cycles : 0;
        return s;
    }

private:
    void finish(Req *r, double now, std::vector<Req *> &finished)
    {
        r->state = kDone;
        r->t_finish = now;
        if (r->status == 0) {
            ++st_.completed;
            st_.work_done += r->work;
            lat_.push_back(now - r->t_submit);
        }
        finished.push_back(r);
    }

    Allocator alloc_;
    int max_active_, quantum_, max_queue_;
    std::deque<Req *> wait_;
    std::vector<Req *> active_;
    std::vector<double> lat_;
    Stats st_;
};

}  // namespace sched
}  // namespace gm
