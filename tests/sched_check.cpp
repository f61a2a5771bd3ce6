// Host-only checks of the serving scheduler (serving_sched.h) with a fake
// executor: no device, no HIP. Built and run by test_serving_sched_cpu.py,
// also under AddressSanitizer + UndefinedBehaviorSanitizer and under
// ThreadSanitizer (the fake executor completes requests from a worker
// thread, as HIP runs stream callbacks on a thread of its own).
//
// Each check prints "ok <name>" or "FAIL <name>: <what>" and the program
// exits non-zero on any failure.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include "../paper_1611_00606_amd/csrc/serving_sched.h"

using hs::serve::ADMIT_BYPASS;
using hs::serve::ADMIT_FIFO;
using hs::serve::ALIGN;
using hs::serve::Arena;
using hs::serve::Request;
using hs::serve::Scheduler;

static int g_fail = 0;
#define CHECK(name, cond, ...)                               \
    do {                                                     \
        if (!(cond)) {                                       \
            std::printf("FAIL %s: ", name);                  \
            std::printf(__VA_ARGS__);                        \
            std::printf("\n");                               \
            ++g_fail;                                        \
            return;                                          \
        }                                                    \
    } while (0)

// Executor whose "device" is one worker thread: started requests run for a
// fixed number of ticks of a virtual clock, then the worker calls finish().
class FakeExec {
   public:
    explicit FakeExec(bool threaded) : threaded_(threaded) {
        if (threaded_) worker_ = std::thread([this] { loop(); });
    }
    ~FakeExec() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
        }
        cv_.notify_all();
        if (worker_.joinable()) worker_.join();
    }
    // start: the request runs for `ticks` calls of tick() (or, threaded,
    // about that many microseconds of the worker).
    int start(Request *r, int ticks) {
        std::lock_guard<std::mutex> lk(mu_);
        running_.push_back({r, ticks});
        cv_.notify_all();
        return 0;
    }
    // unthreaded: one step of the virtual device
    void tick(double now) {
        std::lock_guard<std::mutex> lk(mu_);
        for (auto it = running_.begin(); it != running_.end();) {
            if (--it->second <= 0) {
                it->first->finish(now);
                it = running_.erase(it);
            } else {
                ++it;
            }
        }
    }

   private:
    void loop() {
        std::unique_lock<std::mutex> lk(mu_);
        while (!stop_) {
            if (running_.empty()) {
                cv_.wait(lk);
                continue;
            }
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(50));
            lk.lock();
            for (auto it = running_.begin(); it != running_.end();) {
                if (--it->second <= 0) {
                    it->first->finish(0.0);
                    it = running_.erase(it);
                } else {
                    ++it;
                }
            }
        }
    }
    bool threaded_;
    bool stop_ = false;
    std::mutex mu_;
    std::condition_variable cv_;
    std::deque<std::pair<Request *, int>> running_;
    std::thread worker_;
};

struct Rec : Request {
    int ticks = 1;
    int order = 0;   // arrival index
};

static void arena_invariants() {
    const char *name = "arena_invariants";
    Arena a;
    a.init(1 << 20);
    std::mt19937 rng(7);
    std::vector<std::pair<size_t, size_t>> held;
    for (int step = 0; step < 20000; ++step) {
        if (held.empty() || (rng() % 3 != 0 && held.size() < 64)) {
            const size_t n = 1 + rng() % 40000;
            size_t off;
            if (a.alloc(n, off)) {
                for (auto &h : held)
                    CHECK(name, off + hs::serve::align_up(n) <= h.first || h.first + hs::serve::align_up(h.second) <= off,
                          "block [%zu,+%zu) overlaps [%zu,+%zu)", off, n, h.first, h.second);
                CHECK(name, off % ALIGN == 0 && off + n <= a.size(), "block out of bounds");
                held.push_back({off, n});
            }
        } else {
            const size_t k = rng() % held.size();
            a.release(held[k].first, held[k].second);
            held.erase(held.begin() + k);
        }
        CHECK(name, a.consistent(), "free list inconsistent at step %d", step);
    }
    for (auto &h : held) a.release(h.first, h.second);
    CHECK(name, a.used() == 0 && a.free_blocks() == 1 && a.consistent(),
          "arena not whole after releasing everything (%zu used, %zu blocks)", a.used(),
          a.free_blocks());
    size_t off;
    CHECK(name, a.alloc(a.size(), off) && off == 0, "the whole arena is not allocatable");
    std::printf("ok %s\n", name);
}

// Drives a scheduler to completion; checks budget, slots and order on the way.
struct RunResult {
    std::vector<int> admit_order;   // arrival indices in admission order
    int max_running = 0;
    size_t max_used = 0;
    int max_bypassed = 0;
    bool ok = true;
};

static RunResult drive(Scheduler &s, std::vector<Rec *> &reqs, int n_slots, size_t arena,
                       bool threaded, int arrive_per_step) {
    RunResult out;
    FakeExec ex(threaded);
    size_t next = 0;
    int completed = 0;
    double now = 0.0;
    std::vector<Request *> slot_owner(n_slots, nullptr);   // last request started on each slot
    for (int step = 0; completed < (int)reqs.size() && step < 10000000; ++step) {
        now += 1.0;
        for (int k = 0; k < arrive_per_step && next < reqs.size(); ++k, ++next)
            s.submit(reqs[next], now);
        s.progress(
            [&](Request *r) {
                Rec *q = static_cast<Rec *>(r);
                out.admit_order.push_back(q->order);
                // the slot is free: its previous request has finished
                if (r->slot < 0 || r->slot >= n_slots ||
                    (slot_owner[r->slot] && !slot_owner[r->slot]->done.load()))
                    out.ok = false;
                else
                    slot_owner[r->slot] = r;
                return ex.start(r, q->ticks);
            },
            now);
        out.max_running = std::max(out.max_running, s.running());
        out.max_used = std::max(out.max_used, s.used());
        if (s.used() > arena || !s.arena().consistent()) out.ok = false;
        while (Request *r = s.pop()) {
            Rec *q = static_cast<Rec *>(r);
            out.max_bypassed = std::max(out.max_bypassed, q->bypassed);
            if (r->status != 0 || !r->done.load()) out.ok = false;
            if (s.release(r->id) != r) out.ok = false;
            ++completed;
        }
        if (!threaded) ex.tick(now);
        else std::this_thread::yield();
    }
    if (completed != (int)reqs.size()) out.ok = false;
    return out;
}

static std::vector<Rec *> make_requests(int n, size_t arena, unsigned seed, bool with_big) {
    std::mt19937 rng(seed);
    std::vector<Rec *> v;
    for (int i = 0; i < n; ++i) {
        Rec *r = new Rec;
        r->id = 1000 + i;
        r->order = i;
        // mostly small, some big (about half the arena), a few nearly all of it
        size_t b = arena / 16 + rng() % (arena / 8);
        if (with_big && i % 7 == 3) b = arena / 2 + rng() % (arena / 4);
        if (with_big && i % 29 == 11) b = arena - ALIGN;
        r->bytes = b;
        r->ticks = 1 + (int)(rng() % 20);
        v.push_back(r);
    }
    return v;
}

static void fifo_order_budget_slots(bool threaded) {
    const char *name = threaded ? "fifo_threaded" : "fifo";
    const size_t arena = 64u << 20;
    const int slots = 3;
    Scheduler s(slots, arena);
    auto reqs = make_requests(300, arena, 11, true);
    RunResult r = drive(s, reqs, slots, arena, threaded, 2);
    for (Rec *q : reqs) delete q;
    CHECK(name, r.ok, "budget, slot or completion invariant broken");
    for (size_t i = 0; i < r.admit_order.size(); ++i)
        CHECK(name, r.admit_order[i] == (int)i, "admission %zu took request %d", i, r.admit_order[i]);
    CHECK(name, r.max_running <= slots && r.max_running >= 2, "max running %d", r.max_running);
    CHECK(name, r.max_used <= arena, "used %zu > arena", r.max_used);
    CHECK(name, r.max_bypassed == 0, "a request was bypassed under FIFO");
    CHECK(name, s.pending() == 0 && s.used() == 0, "left %d pending, %zu bytes", s.pending(), s.used());
    std::printf("ok %s\n", name);
}

static void bypass_bounded(bool threaded, int max_bypass) {
    char name[64];
    std::snprintf(name, sizeof(name), "bypass_%d%s", max_bypass, threaded ? "_threaded" : "");
    const size_t arena = 64u << 20;
    const int slots = 4;
    Scheduler s(slots, arena);
    s.set_policy(ADMIT_BYPASS, max_bypass);
    auto reqs = make_requests(300, arena, 12, true);
    RunResult r = drive(s, reqs, slots, arena, threaded, 2);
    for (Rec *q : reqs) delete q;
    CHECK(name, r.ok, "budget, slot or completion invariant broken");
    CHECK(name, r.max_bypassed <= max_bypass, "a request was passed %d times", r.max_bypassed);
    int passes = 0;
    for (size_t i = 1; i < r.admit_order.size(); ++i) passes += r.admit_order[i] < r.admit_order[i - 1];
    if (max_bypass > 0) CHECK(name, passes > 0, "no request was ever passed");
    else CHECK(name, passes == 0, "max_bypass 0 still reordered");
    CHECK(name, s.pending() == 0 && s.used() == 0, "left %d pending, %zu bytes", s.pending(), s.used());
    std::printf("ok %s (%d passes)\n", name, passes);
}

// A head that does not fit blocks FIFO but not BYPASS; BYPASS then lets the
// head in once it has been passed max_bypass times and space frees.
static void head_of_line() {
    const char *name = "head_of_line";
    const size_t arena = 10 * ALIGN * 1024;
    for (int policy : {ADMIT_FIFO, ADMIT_BYPASS}) {
        Scheduler s(4, arena);
        s.set_policy(policy, 2);
        FakeExec ex(false);
        Rec big1, big2, small1, small2, small3;
        big1.id = 1, big1.bytes = arena * 6 / 10, big1.ticks = 5;
        big2.id = 2, big2.bytes = arena * 6 / 10, big2.ticks = 1;
        small1.id = 3, small1.bytes = arena / 10, small1.ticks = 1;
        small2.id = 4, small2.bytes = arena / 10, small2.ticks = 1;
        small3.id = 5, small3.bytes = arena / 10, small3.ticks = 1;
        std::vector<int64_t> admitted;
        auto start = [&](Request *r) {
            admitted.push_back(r->id);
            return ex.start(r, static_cast<Rec *>(r)->ticks);
        };
        for (Rec *r : {&big1, &big2, &small1, &small2, &small3}) s.submit(r, 0.0);
        s.progress(start, 0.0);
        if (policy == ADMIT_FIFO) {
            CHECK(name, admitted.size() == 1 && admitted[0] == 1, "FIFO admitted %zu", admitted.size());
        } else {
            // big2 waits; small1 and small2 pass it (2 = max_bypass), then small3 must wait
            CHECK(name, admitted.size() == 3 && admitted[1] == 3 && admitted[2] == 4,
                  "BYPASS admitted %zu", admitted.size());
            CHECK(name, big2.bypassed == 2, "big2 passed %d times", big2.bypassed);
        }
        int rounds = 0;
        while (s.pending() && rounds++ < 100) {
            ex.tick(1.0 + rounds);
            s.progress(start, 1.0 + rounds);
            while (Request *r = s.pop()) s.release(r->id);
        }
        CHECK(name, s.pending() == 0 && s.used() == 0, "policy %d did not drain", policy);
        CHECK(name, admitted.size() == 5, "policy %d admitted %zu", policy, admitted.size());
        const auto pos2 = std::find(admitted.begin(), admitted.end(), (int64_t)2) - admitted.begin();
        const auto pos5 = std::find(admitted.begin(), admitted.end(), (int64_t)5) - admitted.begin();
        CHECK(name, pos2 < pos5, "policy %d: the passed head started after a later request", policy);
    }
    std::printf("ok %s\n", name);
}

// A start that fails completes at once with its status and frees its space.
static void failed_start() {
    const char *name = "failed_start";
    Scheduler s(2, 1 << 20);
    Rec a, b;
    a.id = 1, a.bytes = 4096;
    b.id = 2, b.bytes = 4096;
    s.submit(&a, 0.0);
    s.submit(&b, 0.0);
    int n = s.progress([&](Request *r) { return r->id == 1 ? 7 : 0; }, 0.0);
    CHECK(name, n == 1, "%d results ready", n);
    Request *r = s.pop();
    CHECK(name, r == &a && r->status == 7 && r->done.load(), "failed request not reported");
    CHECK(name, s.release(1) == &a, "release");
    CHECK(name, s.running() == 1 && s.used() == hs::serve::align_up(4096), "slot or space not freed");
    b.finish(1.0);
    s.progress([](Request *) { return 0; }, 1.0);
    CHECK(name, s.pop() == &b && s.release(2) == &b && s.used() == 0, "second request");
    CHECK(name, s.release(99) == nullptr, "release of an unknown id");
    std::printf("ok %s\n", name);
}

static void oversize() {
    const char *name = "oversize";
    Scheduler s(1, 1 << 20);
    CHECK(name, s.fits_ever(1 << 20) && !s.fits_ever((1 << 20) + 1), "fits_ever bound");
    Arena a;
    a.init(1000);   // rounded down to whole blocks
    CHECK(name, a.size() == 768 && !a.fits_ever(769) && a.fits_ever(768), "arena rounding");
    std::printf("ok %s\n", name);
}

int main() {
    arena_invariants();
    oversize();
    failed_start();
    head_of_line();
    fifo_order_budget_slots(false);
    fifo_order_budget_slots(true);
    bypass_bounded(false, 0);
    bypass_bounded(false, 3);
    bypass_bounded(true, 3);
    if (g_fail) {
        std::printf("%d check(s) failed\n", g_fail);
        return 1;
    }
    std::printf("all scheduler checks passed\n");
    return 0;
}
