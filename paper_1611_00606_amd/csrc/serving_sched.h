// Host-side scheduling of the serving loop, independent of the device: a
// first-fit arena over byte offsets, and the admission and completion
// bookkeeping of requests over a fixed number of slots (one k-point build
// per slot at a time). The executor - the HIP one in hs_serving.hip, or a
// fake one in the CPU tests - starts an admitted request and later marks it
// done, possibly from another thread (HIP runs stream callbacks on a thread
// of its own), through Request::finish.
//
// Admission policies:
//   ADMIT_FIFO    requests start in arrival order; a request whose footprint
//                 does not fit the free arena holds back every later one
//                 (head-of-line blocking).
//   ADMIT_BYPASS  a later request that fits may start while an earlier one
//                 waits for arena space; each start that passes a waiting
//                 request counts against it, and once a waiting request has
//                 been passed max_bypass times nothing behind it starts until
//                 it has (bounded waiting: no request starves).
#pragma once

#include <atomic>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <iterator>
#include <map>
#include <unordered_map>
#include <vector>

namespace hs {
namespace serve {

constexpr size_t ALIGN = 256;
inline size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

enum { ADMIT_FIFO = 0, ADMIT_BYPASS = 1 };

// First-fit allocator over [0, size) with a coalescing free list (offset ->
// length); every block is a multiple of ALIGN bytes.
class Arena {
   public:
    void init(size_t size) {
        free_.clear();
        size_ = size / ALIGN * ALIGN;
        if (size_) free_[0] = size_;
        used_ = 0;
    }
    bool alloc(size_t n, size_t &off) {
        n = align_up(n);
        if (n == 0) n = ALIGN;
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
    void release(size_t off, size_t n) {
        n = align_up(n);
        if (n == 0) n = ALIGN;
        used_ -= n;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }
    size_t size() const { return size_; }
    // Whether a block of n bytes can ever be held (an empty arena fits it).
    bool fits_ever(size_t n) const { return align_up(n == 0 ? 1 : n) <= size_; }
    // Invariants: free blocks in bounds, ordered, disjoint and never adjacent
    // (coalesced); free + used = size.
    bool consistent() const {
        size_t end = 0, total = 0;
        bool first = true;
        for (const auto &kv : free_) {
            if (kv.second == 0 || kv.first % ALIGN || kv.second % ALIGN) return false;
            if (!first && kv.first <= end) return false;   // overlap or adjacency
            end = kv.first + kv.second;
            if (end > size_) return false;
            total += kv.second;
            first = false;
        }
        return total + used_ == size_;
    }
    size_t free_blocks() const { return free_.size(); }

   private:
    std::map<size_t, size_t> free_;
    size_t size_ = 0, used_ = 0;
};

// One request's scheduling state. The executor derives its own record from
// it; the scheduler only reads and writes these fields.
struct Request {
    int64_t id = 0;
    size_t bytes = 0;      // device footprint
    size_t off = 0;        // arena offset once admitted
    int slot = -1;         // slot while running, -1 before admission
    int status = 0;        // 0, or the executor's error status
    int bypassed = 0;      // later requests started while this one waited
    double t_submit = 0, t_admit = 0;
    std::atomic<double> t_done{0.0};
    std::atomic<int> done{0};
    virtual ~Request() = default;
    // Called by the executor (any thread) when the request's work has ended.
    void finish(double t) {
        t_done.store(t, std::memory_order_relaxed);
        done.store(1, std::memory_order_release);
    }
};

class Scheduler {
   public:
    Scheduler(int n_slots, size_t arena_bytes) : slots_(n_slots, nullptr) { arena_.init(arena_bytes); }

    void set_policy(int policy, int max_bypass) {
        policy_ = policy;
        max_bypass_ = max_bypass < 0 ? 0 : max_bypass;
    }
    int policy() const { return policy_; }
    bool fits_ever(size_t bytes) const { return arena_.fits_ever(bytes); }

    void submit(Request *r, double now) {
        r->t_submit = now;
        queue_.push_back(r);
    }

    // Collects completions, then admits what the policy allows. start(r)
    // begins the work of an admitted request (r->off, r->slot set) and
    // returns 0, or an error status after making sure nothing it began is
    // still running; the request then completes at once with that status.
    // Returns the number of completed results waiting to be popped.
    template <class Start>
    int progress(Start &&start, double now) {
        for (auto &s : slots_) {
            if (s && s->done.load(std::memory_order_acquire)) {
                done_.push_back(s);
                s = nullptr;
            }
        }
        for (auto it = queue_.begin(); it != queue_.end();) {
            const int slot = free_slot();
            if (slot < 0) break;
            Request *r = *it;
            // starting r passes every request still waiting ahead of it:
            // not allowed once one of them has been passed max_bypass times
            bool blocked = false;
            for (auto jt = queue_.begin(); jt != it; ++jt) blocked |= (*jt)->bypassed >= max_bypass_;
            if (blocked) break;
            size_t off = 0;
            if (!arena_.alloc(r->bytes, off)) {
                if (policy_ == ADMIT_FIFO || r->bypassed >= max_bypass_) break;
                ++it;
                continue;
            }
            for (auto jt = queue_.begin(); jt != it; ++jt) ++(*jt)->bypassed;
            it = queue_.erase(it);
            r->off = off;
            r->slot = slot;
            r->t_admit = now;
            slots_[slot] = r;
            const int rc = start(r);
            if (rc != 0) {
                slots_[slot] = nullptr;
                r->status = rc;
                r->finish(now);
                done_.push_back(r);
            }
        }
        return (int)done_.size();
    }

    // Oldest completed request (now held until release), or nullptr.
    Request *pop() {
        if (done_.empty()) return nullptr;
        Request *r = done_.front();
        done_.pop_front();
        popped_[r->id] = r;
        return r;
    }

    // Frees a popped request's arena space and hands the record back to the
    // caller (nullptr if no popped request has this id).
    Request *release(int64_t id) {
        auto it = popped_.find(id);
        if (it == popped_.end()) return nullptr;
        Request *r = it->second;
        popped_.erase(it);
        if (r->slot >= 0) arena_.release(r->off, r->bytes);
        return r;
    }

    int pending() const {
        int n = (int)queue_.size() + (int)done_.size();
        for (Request *s : slots_) n += s != nullptr;
        return n;
    }
    size_t used() const { return arena_.used(); }
    const Arena &arena() const { return arena_; }
    int running() const {
        int n = 0;
        for (Request *s : slots_) n += s != nullptr;
        return n;
    }

    // Every record the scheduler still refers to (for teardown).
    template <class F>
    void for_each(F &&f) const {
        for (Request *r : slots_)
            if (r) f(r);
        for (Request *r : queue_) f(r);
        for (Request *r : done_) f(r);
        for (const auto &kv : popped_) f(kv.second);
    }

   private:
    int free_slot() const {
        for (size_t i = 0; i < slots_.size(); ++i)
            if (!slots_[i]) return (int)i;
        return -1;
    }

    Arena arena_;
    std::vector<Request *> slots_;
    std::deque<Request *> queue_;                    // submitted, not admitted
    std::deque<Request *> done_;                     // completed, not popped
    std::unordered_map<int64_t, Request *> popped_;  // popped, not released
    int policy_ = ADMIT_FIFO;
    int max_bypass_ = 0;
};

}  // namespace serve
}  // namespace hs
