// Host check of the served-request admission (csrc/admission.h) against a
// simulated executor: requests of seeded random sizes arrive over time, run
// a random number of ticks once admitted, and release their memory when
// done.  Checked at every tick: admission in submission order, the
// max_active bound, allocations disjoint and inside the budget, the
// reserved bytes equal to the arena's count, and no idle slot while the
// oldest pending request fits.  At the end every request has run and the
// arena is one free block again.  Prints "ok" or the first violation.
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <random>
#include <vector>

#include "admission.h"

struct Req {
    size_t bytes = 0, off = (size_t)-1;
    int id = 0, left = 0;
};

static int fail(const char* what, int tick) {
    std::printf("violation at tick %d: %s\n", tick, what);
    return 1;
}

int run(unsigned seed, size_t budget, int max_active, int count) {
    std::mt19937_64 rng(seed);
    std::uniform_int_distribution<size_t> size(1, budget / 3);
    std::uniform_int_distribution<int> ticks(1, 12), arrive(0, 3);
    std::vector<Req> reqs(count);
    for (int i = 0; i < count; ++i) {
        reqs[i].id = i;
        reqs[i].bytes = size(rng);
        reqs[i].left = ticks(rng);
    }
    adi::Arena arena;
    arena.reset(budget);
    std::deque<Req*> pending;
    std::vector<Req*> active;
    int next = 0, admitted_order = 0, done = 0;
    for (int tick = 0; done < count; ++tick) {
        if (tick > 100000) return fail("no progress", tick);
        for (int a = arrive(rng); a > 0 && next < count; --a) pending.push_back(&reqs[next++]);
        // admit while the rule allows (the uploader's loop)
        while (adi::admissible(pending, (int64_t)active.size(), max_active, arena)) {
            Req* r = pending.front();
            pending.pop_front();
            if (r->id != admitted_order++) return fail("admission out of submission order", tick);
            active.push_back(r);
        }
        if ((int)active.size() > max_active) return fail("more than max_active admitted", tick);
        // reservations: disjoint, inside the budget, counted by the arena
        std::vector<std::pair<size_t, size_t>> iv;
        for (Req* r : active) iv.push_back({r->off, (r->bytes + 255) / 256 * 256});
        if (!pending.empty() && pending.front()->off != (size_t)-1)
            iv.push_back({pending.front()->off, (pending.front()->bytes + 255) / 256 * 256});
        size_t sum = 0;
        for (size_t i = 0; i < iv.size(); ++i) {
            if (iv[i].first % 256 || iv[i].first + iv[i].second > budget) return fail("block outside the budget", tick);
            sum += iv[i].second;
            for (size_t j = 0; j < i; ++j)
                if (iv[i].first < iv[j].first + iv[j].second && iv[j].first < iv[i].first + iv[i].second)
                    return fail("overlapping blocks", tick);
        }
        if (sum != arena.used()) return fail("reserved bytes differ from the arena's count", tick);
        // liveness: an idle slot with a pending request means it does not fit
        if (!pending.empty() && (int)active.size() < max_active) {
            if (pending.front()->off != (size_t)-1) return fail("reserved request left waiting", tick);
            size_t largest = 0;
            for (const auto& kv : arena.free_blocks()) largest = kv.second > largest ? kv.second : largest;
            if (largest >= (pending.front()->bytes + 255) / 256 * 256) return fail("fitting request not admitted", tick);
        }
        // one tick of the executor
        std::vector<Req*> keep;
        for (Req* r : active) {
            if (--r->left == 0) {
                arena.release(r->off, r->bytes);
                ++done;
            } else {
                keep.push_back(r);
            }
        }
        active.swap(keep);
    }
    if (arena.used() != 0) return fail("memory left reserved", -1);
    if (arena.free_blocks().size() != 1 || arena.free_blocks().begin()->first != 0 ||
        arena.free_blocks().begin()->second != budget)
        return fail("free list not coalesced into one block", -1);
    return 0;
}

int main() {
    const size_t budgets[3] = {(size_t)1 << 20, (size_t)64 << 20, (size_t)1 << 30};
    const int actives[3] = {1, 4, 64};
    for (unsigned seed = 0; seed < 20; ++seed)
        for (size_t b : budgets)
            for (int m : actives)
                if (run(seed, b, m, 400)) {
                    std::printf("seed %u budget %zu max_active %d\n", seed, b, m);
                    return 1;
                }
    std::printf("ok\n");
    return 0;
}
