// Host-only checks of the serving scheduler pieces (sched.hpp) with a fake
// executor and a fake clock: a discrete-event simulation of requests that
// arrive, are admitted into slots and device memory, run for a service time
// and complete.  Exits non-zero on the first violated property.
//
//   arena      random alloc / free: no overlap, used() exact, full coalescing
//   percentile nearest-rank values on known data
//   mixed      random mix near saturation: memory and slot limits hold at
//              every step; a request is admitted ahead of an older waiting
//              one only when that one was offered in the same pass and did
//              not fit; every request completes
//   starvation a large request behind a steady stream of small ones runs
//              after a bounded wait; with the head rule disabled only once
//              the stream has stopped
//   sizeaware  the default order (aged requests first, oldest first, then
//              ascending cost) with at most one large request in flight:
//              the queue is in that order before every pass, the cap and
//              the memory and slot limits hold, every request completes,
//              no request waits much beyond the aging bound plus one large
//              service, and small requests wait less than in arrival order
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <vector>

#include "sched.hpp"

using stk::Arena;

static int fail(const char* what) {
    std::printf("FAIL: %s\n", what);
    return 1;
}

static int test_arena() {
    const size_t units = 4096, size = units * 256;
    Arena a(size);
    std::mt19937_64 rng(1);
    struct Live { size_t off, bytes; };
    std::vector<Live> live;
    for (int step = 0; step < 20000; ++step) {
        if (live.empty() || rng() % 3 != 0) {
            const size_t bytes = 1 + rng() % (64 * 256);
            size_t off;
            if (a.alloc(bytes, &off)) {
                const size_t r = (bytes + 255) / 256 * 256;
                if (off % 256 || off + r > size) return fail("arena: range outside the arena");
                for (const Live& l : live) {
                    const size_t lr = (l.bytes + 255) / 256 * 256;
                    if (off < l.off + lr && l.off < off + r) return fail("arena: overlapping ranges");
                }
                live.push_back({off, bytes});
            }
        } else {
            const size_t i = rng() % live.size();
            a.free(live[i].off, live[i].bytes);
            live.erase(live.begin() + (long)i);
        }
        size_t used = 0;
        for (const Live& l : live) used += (l.bytes + 255) / 256 * 256;
        if (used != a.used()) return fail("arena: used() differs from the live ranges");
    }
    for (const Live& l : live) a.free(l.off, l.bytes);
    if (a.used() != 0 || a.largest_free() != size) return fail("arena: freeing everything does not coalesce");
    std::printf("arena ok\n");
    return 0;
}

static int test_percentile() {
    std::vector<double> v;
    if (stk::nearest_rank(v, 0.5) != 0.0) return fail("percentile: empty");
    v = {5.0};
    if (stk::nearest_rank(v, 0.5) != 5.0 || stk::nearest_rank(v, 0.99) != 5.0) return fail("percentile: one value");
    v = {1.0, 2.0};
    if (stk::nearest_rank(v, 0.5) != 1.0 || stk::nearest_rank(v, 0.99) != 2.0) return fail("percentile: two values");
    v.clear();
    for (int i = 1; i <= 100; ++i) v.push_back(i);
    if (stk::nearest_rank(v, 0.5) != 50.0 || stk::nearest_rank(v, 0.99) != 99.0 || stk::nearest_rank(v, 1.0) != 100.0)
        return fail("percentile: 1..100");
    v.clear();
    for (int i = 1; i <= 1000; ++i) v.push_back(i);
    if (stk::nearest_rank(v, 0.99) != 990.0) return fail("percentile: 1..1000");
    std::printf("percentile ok\n");
    return 0;
}

struct Req {
    int id;
    size_t bytes;
    double arrive, service;
    double admit = -1, done = -1;
    size_t off = 0;
    int passed = 0;
};

struct SimResult {
    int completed = 0, total = 0;
    double max_wait = 0, large_wait = -1;
    bool ok = true;
    const char* why = "";
};

// Discrete-time simulation (step dt).  `reqs` in arrival order.
static SimResult simulate(std::vector<Req>& reqs, size_t budget, int slots, double dt, double t_end,
                          int max_pass, int max_head_passes, int large_id) {
    SimResult r;
    r.total = (int)reqs.size();
    Arena arena(budget);
    std::deque<Req*> waiting;
    std::vector<Req*> running;
    size_t next = 0;
    for (double now = 0; now < t_end; now += dt) {
        for (auto it = running.begin(); it != running.end();) {   // completions
            if ((*it)->admit + (*it)->service <= now) {
                (*it)->done = now;
                arena.free((*it)->off, (*it)->bytes);
                ++r.completed;
                it = running.erase(it);
            } else {
                ++it;
            }
        }
        while (next < reqs.size() && reqs[next].arrive <= now) waiting.push_back(&reqs[next++]);
        std::set<int> offered;   // requests offered in this pass that did not fit
        auto slot_free = [&] { return (int)running.size() < slots; };
        auto take = [&](Req* q) {
            size_t off;
            if (!arena.alloc(q->bytes, &off)) {
                offered.insert(q->id);
                return false;
            }
            for (Req* w : waiting)   // every older waiting request was offered and did not fit
                if (w->id < q->id && !offered.count(w->id)) {
                    r.ok = false;
                    r.why = "a younger request was admitted past an older one that was not offered";
                }
            q->off = off;
            q->admit = now;
            r.max_wait = std::max(r.max_wait, now - q->arrive);
            running.push_back(q);
            return true;
        };
        stk::admission_pass(waiting, slot_free, take, max_pass, max_head_passes);
        if (arena.used() > budget) { r.ok = false; r.why = "memory budget exceeded"; }
        if ((int)running.size() > slots) { r.ok = false; r.why = "more requests than slots"; }
        if (!r.ok) return r;
        if (next == reqs.size() && waiting.empty() && running.empty()) break;
    }
    if (large_id >= 0 && reqs[large_id].admit >= 0) r.large_wait = reqs[large_id].admit - reqs[large_id].arrive;
    return r;
}

static int test_mixed() {
    std::mt19937_64 rng(7);
    std::vector<Req> reqs;
    double t = 0;
    const size_t unit = 256 * 1024;
    for (int i = 0; i < 3000; ++i) {
        t += std::exponential_distribution<double>(1.0)(rng);
        const bool large = rng() % 100 < 15;
        const size_t units = large ? 300 + rng() % 600 : 10 + rng() % 40;
        reqs.push_back({i, units * unit, t, 0.004 * (double)units});
    }
    SimResult r = simulate(reqs, 1000 * unit, 4, 0.01, 1e6, 8, 1000, -1);
    if (!r.ok) return fail(r.why);
    if (r.completed != r.total) return fail("mixed: not every request completed");
    std::printf("mixed ok: %d requests, longest wait %.1f\n", r.completed, r.max_wait);
    return 0;
}

static int test_starvation() {
    // a steady stream of small requests (from t = 0, one every 0.25, each
    // running 1.0 and holding 60 of 1000 units) keeps 180-240 units in use;
    // a large request of 900 units arrives at t = 0.6 and never finds room
    // unless the stream stops overtaking it
    const size_t unit = 256 * 1024;
    int large = -1;
    auto make = [&] {
        std::vector<Req> reqs;
        for (double t = 0.0; t < 2000.0; t += 0.25) {
            if (t > 0.6 && t - 0.25 < 0.6) {
                large = (int)reqs.size();
                reqs.push_back({large, 900 * unit, 0.6, 1.0});
            }
            reqs.push_back({(int)reqs.size(), 60 * unit, t, 1.0});
        }
        return reqs;
    };
    std::vector<Req> with_rule = make();
    SimResult r = simulate(with_rule, 1000 * unit, 8, 0.05, 2100.0, 8, 200, large);
    if (!r.ok) return fail(r.why);
    if (with_rule[large].done < 0) return fail("starvation: the large request never ran");
    if (r.completed != r.total) return fail("starvation: not every request completed");
    std::vector<Req> without = make();
    SimResult r0 = simulate(without, 1000 * unit, 8, 0.05, 2100.0, 8, 1 << 30, large);
    if (!r0.ok) return fail(r0.why);
    if (r.large_wait > 50.0) return fail("starvation: the large request waited too long with the head rule");
    // without the rule it runs only once the stream has stopped
    if (without[large].admit >= 0 && without[large].admit < 1999.0)
        return fail("starvation: the scenario does not starve without the head rule");
    std::printf("starvation ok: large request admitted after %.1f with the head rule, after %.1f without\n",
                r.large_wait, without[large].admit - without[large].arrive);
    return 0;
}

// Cost-aware simulation: service time doubles as the modelled cost; the
// queue is ordered by order_waiting before every pass (fifo: not at all) and
// large requests (cost >= large.threshold) are capped by `large`.
struct PolicyResult {
    bool ok = true;
    const char* why = "";
    int completed = 0;
    double small_wait = 0, max_wait = 0, max_aged_wait = 0;
};

static PolicyResult simulate_policy(std::vector<Req>& reqs, size_t budget, int slots, double dt, double aging,
                                    stk::LargeCap large, bool fifo) {
    PolicyResult r;
    Arena arena(budget);
    std::deque<Req*> waiting;
    std::vector<Req*> running;
    size_t next = 0;
    int nsmall = 0;
    auto arrival = [](const Req* q) { return q->arrive; };
    auto cost = [](const Req* q) { return q->service; };
    for (double now = 0; now < 1e7; now += dt) {
        for (auto it = running.begin(); it != running.end();) {
            if ((*it)->admit + (*it)->service <= now) {
                (*it)->done = now;
                arena.free((*it)->off, (*it)->bytes);
                if (large.large((*it)->service)) --large.inflight;
                ++r.completed;
                it = running.erase(it);
            } else {
                ++it;
            }
        }
        while (next < reqs.size() && reqs[next].arrive <= now) waiting.push_back(&reqs[next++]);
        if (!fifo) {
            stk::order_waiting(waiting, now, aging, arrival, cost);
            for (size_t i = 1; i < waiting.size(); ++i) {   // aged first (oldest first), then by cost
                const Req *a = waiting[i - 1], *b = waiting[i];
                const bool oa = now - a->arrive > aging, ob = now - b->arrive > aging;
                if ((!oa && ob) || (oa && ob && a->arrive > b->arrive) || (!oa && !ob && a->service > b->service)) {
                    r.ok = false;
                    r.why = "sizeaware: queue not in the size-aware order";
                    return r;
                }
            }
        }
        auto slot_free = [&] { return (int)running.size() < slots; };
        auto take = [&](Req* q) {
            if (!fifo && !large.admits(q->service)) return false;
            size_t off;
            if (!arena.alloc(q->bytes, &off)) return false;
            q->off = off;
            q->admit = now;
            if (large.large(q->service)) ++large.inflight;
            const double w = now - q->arrive;
            r.max_wait = std::max(r.max_wait, w);
            if (!large.large(q->service)) { r.small_wait += w; ++nsmall; }
            running.push_back(q);
            return true;
        };
        stk::admission_pass(waiting, slot_free, take, 8, 1000);
        if (arena.used() > budget) { r.ok = false; r.why = "sizeaware: memory budget exceeded"; }
        if ((int)running.size() > slots) { r.ok = false; r.why = "sizeaware: more requests than slots"; }
        if (!fifo && large.inflight > large.cap) { r.ok = false; r.why = "sizeaware: large-request cap exceeded"; }
        if (!r.ok) return r;
        if (next == reqs.size() && waiting.empty() && running.empty()) break;
    }
    if (nsmall) r.small_wait /= nsmall;
    return r;
}

static int test_size_aware() {
    // heavy-tailed service times: small requests log-uniform over
    // 0.01 .. 1, about 3 % large ones over 1 .. 3; four slots about 70 %
    // busy, the large requests alone about 55 % of one slot (their queue is
    // stable with the cap of one)
    auto make = [] {
        std::mt19937_64 rng(11);
        std::vector<Req> reqs;
        double t = 0;
        const size_t unit = 256 * 1024;
        std::uniform_real_distribution<double> u(0.0, 1.0);
        for (int i = 0; i < 3000; ++i) {
            t += std::exponential_distribution<double>(10.8)(rng);
            const bool large = u(rng) < 0.028;
            const double lo = large ? 1.0 : 0.01, hi = large ? 3.0 : 1.0;
            const double svc = std::exp(std::log(lo) + u(rng) * (std::log(hi) - std::log(lo)));
            reqs.push_back({i, (size_t)(1 + svc * 60) * unit, t, svc});
        }
        return reqs;
    };
    stk::LargeCap cap;
    cap.threshold = 1.0;
    cap.cap = 1;
    const double aging = 5.0;
    std::vector<Req> sa = make(), ff = make();
    PolicyResult a = simulate_policy(sa, 1000 * 256 * 1024, 4, 0.01, aging, cap, false);
    if (!a.ok) return fail(a.why);
    PolicyResult f = simulate_policy(ff, 1000 * 256 * 1024, 4, 0.01, aging, cap, true);
    if (!f.ok) return fail(f.why);
    if (a.completed != (int)sa.size() || f.completed != (int)ff.size()) return fail("sizeaware: not every request completed");
    // a request waits at most the aging bound, then behind the older aged
    // requests and (large ones) behind the one large request in flight
    double longest = 0;
    for (const Req& q : sa) longest = std::max(longest, q.service);
    if (a.max_wait > 3 * (aging + longest)) return fail("sizeaware: a request waited far beyond the aging bound");
    if (!(a.small_wait < f.small_wait)) return fail("sizeaware: small requests do not wait less than in arrival order");
    std::printf("sizeaware ok: mean small-request wait %.3f (arrival order %.3f), longest wait %.2f (aging %.1f)\n",
                a.small_wait, f.small_wait, a.max_wait, aging);
    return 0;
}

int main() {
    int rc = 0;
    rc |= test_arena();
    rc |= test_percentile();
    rc |= test_mixed();
    rc |= test_starvation();
    rc |= test_size_aware();
    if (rc == 0) std::printf("all ok\n");
    return rc;
}
