// Host-only checks of the serving loop's admission policy (mg_sched.h) with a
// mock device backend and a simulated clock.  Prints one line per scenario and
// exits non-zero on the first violated property.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <map>
#include <set>
#include <vector>

#include "mg_sched.h"

namespace {

struct Hier {
    int dim, n;
    size_t bytes;
};

struct MockBackend {
    size_t capacity = SIZE_MAX;  // device memory; alloc answers "out of memory" beyond it
    size_t live = 0;             // bytes held by hierarchies that exist
    int allocs = 0, releases = 0;
    bool fail = false;  // report a device error on the next alloc
    std::set<Hier*> alive;
    size_t bytes(int dim, int n) const {
        const size_t p = dim == 2 ? (size_t)n * n : (size_t)n * n * n;
        return p * 28 + 4096;
    }
    size_t bytes_of(const Hier* h) const { return h->bytes; }
    int alloc(int dim, int n, Hier** out) {
        if (fail) return -4;
        const size_t b = bytes(dim, n);
        if (live + b > capacity) return 1;
        *out = new Hier{dim, n, b};
        live += b;
        ++allocs;
        alive.insert(*out);
        return 0;
    }
    void release(Hier* h) {
        live -= h->bytes;
        ++releases;
        alive.erase(h);
        delete h;
    }
};

// splitmix64, for the simulated arrival stream
struct Rng {
    uint64_t s;
    uint64_t next() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    double uni() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
};

int g_fail = 0;
#define CHECK(cond, ...)                                   \
    do {                                                   \
        if (!(cond)) {                                     \
            std::printf("FAIL %s:%d: ", __FILE__, __LINE__); \
            std::printf(__VA_ARGS__);                      \
            std::printf("\n");                             \
            g_fail = 1;                                    \
            return false;                                  \
        }                                                  \
    } while (0)

struct Req {
    long long id;
    int dim, n;
    double arrive;
    double admitted = -1, done = -1;
    int slot = -1;
    Hier* h = nullptr;
};

// Run an arrival stream through the policy.  Each admitted request runs for a
// time proportional to its size.  Checks budget, slots, arrival-order
// admission, memory accounting and completion of every request.
bool simulate(const char* name, uint64_t seed, int count, double rate, size_t budget, int slots, size_t capacity,
              bool expect_no_release) {
    Rng rng{seed};
    const int e2[4] = {257, 513, 1025, 2049}, e3[4] = {33, 65, 129, 257};
    std::vector<Req> reqs;
    double t = 0.0;
    MockBackend b;
    b.capacity = capacity;
    mg::Sched<Hier*> S;
    S.init(budget, slots);
    for (int i = 0; i < count; ++i) {
        t += -std::log(1.0 - rng.uni()) / rate;
        const bool two = rng.uni() < 0.6;
        const int e = (int)(rng.uni() * 4) & 3;
        reqs.push_back(Req{i + 1, two ? 2 : 3, two ? e2[e] : e3[e], t});
        CHECK(b.bytes(reqs.back().dim, reqs.back().n) <= budget, "request larger than the budget in the stream");
    }
    std::vector<long long> admitted_order;
    size_t next_arrival = 0;
    double now = 0.0;
    std::vector<Req*> running;
    int completed = 0;
    for (int iter = 0; completed < count; ++iter) {
        CHECK(iter < 10000000, "%s: no progress", name);
        while (next_arrival < reqs.size() && reqs[next_arrival].arrive <= now) S.submit(reqs[next_arrival++].id);
        // admit as many as allowed
        while (!S.queue.empty()) {
            Req& r = reqs[(size_t)S.queue.front() - 1];
            int slot = -1;
            Hier* h = nullptr;
            const int a = S.admit_head(b, r.dim, r.n, &slot, &h);
            CHECK(a >= 0, "%s: backend error surfaced without an injected failure", name);
            if (a == 0) break;
            CHECK(h && h->dim == r.dim && h->n == r.n, "%s: hierarchy of the wrong edge", name);
            CHECK(slot >= 0 && slot < slots, "%s: slot out of range", name);
            for (Req* o : running) CHECK(!(o->dim == r.dim && o->slot == slot), "%s: slot given twice", name);
            r.slot = slot;
            r.h = h;
            r.admitted = now;
            running.push_back(&r);
            admitted_order.push_back(r.id);
        }
        CHECK(S.used <= budget, "%s: used %zu > budget %zu", name, S.used, budget);
        CHECK(S.used == b.live, "%s: accounting %zu != live %zu", name, S.used, b.live);
        CHECK(S.active == (int)running.size(), "%s: active count", name);
        int per[2] = {0, 0};
        for (Req* o : running) ++per[o->dim - 2];
        CHECK(per[0] <= slots && per[1] <= slots, "%s: more active than slots", name);
        // advance the clock to the next event (arrival or completion)
        double next = 1e300;
        if (next_arrival < reqs.size()) next = reqs[next_arrival].arrive;
        for (Req* o : running) {
            const double dur = 1e-9 * (double)(o->dim == 2 ? (size_t)o->n * o->n : (size_t)o->n * o->n * o->n);
            if (o->admitted + dur < next) next = o->admitted + dur;
        }
        if (next == 1e300) {
            CHECK(S.queue.empty() && running.empty(), "%s: stalled with %zu queued", name, S.queue.size());
            break;
        }
        now = next;
        std::vector<Req*> keep;
        for (Req* o : running) {
            const double dur = 1e-9 * (double)(o->dim == 2 ? (size_t)o->n * o->n : (size_t)o->n * o->n * o->n);
            if (o->admitted + dur <= now) {
                o->done = now;
                S.retire(o->dim, o->slot, o->n, o->h);
                ++completed;
            } else {
                keep.push_back(o);
            }
        }
        running.swap(keep);
    }
    CHECK(completed == count, "%s: %d of %d completed", name, completed, count);
    for (size_t i = 0; i < admitted_order.size(); ++i)
        CHECK(admitted_order[i] == (long long)i + 1, "%s: request %lld admitted out of arrival order", name,
              admitted_order[i]);
    if (expect_no_release) CHECK(b.releases == 0, "%s: released pooled memory without need", name);
    const int allocs = b.allocs, releases = b.releases;
    S.drain_pool(b);
    CHECK(S.used == 0 && b.live == 0 && b.alive.empty(), "%s: memory left after draining the pool", name);
    std::printf("ok %s: %d requests, %d allocations, %d releases\n", name, count, allocs, releases);
    return true;
}

// Deterministic cases: reuse, eviction, waiting on a full budget, device
// out-of-memory, device error.
bool cases() {
    MockBackend b;
    mg::Sched<Hier*> S;
    const size_t big = b.bytes(3, 257), small = b.bytes(2, 257);
    S.init(big + small, 4);
    int slot;
    Hier* h;
    // 1. admit a 3D 257 and a 2D 257; a second 2D 257 waits for the budget
    S.submit(1);
    S.submit(2);
    S.submit(3);
    CHECK(S.admit_head(b, 3, 257, &slot, &h) == 1 && slot == 0, "admit first");
    Hier* h1 = h;
    CHECK(S.admit_head(b, 2, 257, &slot, &h) == 1 && slot == 0, "admit second");
    Hier* h2 = h;
    CHECK(S.admit_head(b, 2, 257, &slot, &h) == 0 && S.queue.size() == 1, "third must wait (budget)");
    // 2. retiring the 2D request lets the third reuse its hierarchy without allocating
    S.retire(2, 0, 257, h2);
    const int a0 = b.allocs;
    CHECK(S.admit_head(b, 2, 257, &slot, &h) == 1 && h == h2 && b.allocs == a0, "reuse pooled hierarchy");
    S.retire(2, slot, 257, h);
    // 3. a request of another edge evicts the pooled 2D 257 hierarchy only when it must
    S.retire(3, 0, 257, h1);
    S.submit(4);
    CHECK(S.admit_head(b, 2, 513, &slot, &h) == 1, "admit after eviction");
    CHECK(b.releases >= 1 && S.used <= S.budget, "eviction happened and the budget holds");
    S.retire(2, slot, 513, h);
    // 4. device out of memory: the head waits and is admitted once memory frees
    MockBackend tight;
    tight.capacity = tight.bytes(2, 513);
    mg::Sched<Hier*> T;
    T.init(SIZE_MAX / 2, 4);
    T.submit(10);
    T.submit(11);
    CHECK(T.admit_head(tight, 2, 513, &slot, &h) == 1, "oom case: first fits");
    Hier* ht = h;
    CHECK(T.admit_head(tight, 2, 257, &slot, &h) == 0 && T.queue.front() == 11, "oom case: second waits");
    T.retire(2, 0, 513, ht);
    // the pooled 513 fits the budget but not the device: it is released for the 257
    const int r0 = tight.releases;
    CHECK(T.admit_head(tight, 2, 257, &slot, &h) == 1 && tight.releases == r0 + 1,
          "oom case: pooled hierarchy given back when the device is short");
    CHECK(T.used == tight.live, "oom case: accounting");
    T.retire(2, slot, 257, h);
    T.drain_pool(tight);
    // 5. a device error is reported, not swallowed
    tight.fail = true;
    T.submit(12);
    CHECK(T.admit_head(tight, 3, 33, &slot, &h) < 0 && T.queue.size() == 1, "device error surfaces");
    // 6. slots: a dimension with every slot busy waits even with memory to spare
    MockBackend roomy;
    mg::Sched<Hier*> U;
    U.init(SIZE_MAX / 2, 2);
    for (int i = 0; i < 3; ++i) U.submit(20 + i);
    CHECK(U.admit_head(roomy, 3, 33, &slot, &h) == 1, "slot 0");
    CHECK(U.admit_head(roomy, 3, 33, &slot, &h) == 1, "slot 1");
    CHECK(U.admit_head(roomy, 3, 33, &slot, &h) == 0, "no third 3D slot");
    CHECK(U.free_slot(2) == 0, "2D slots are independent");
    S.drain_pool(b);
    std::printf("ok cases\n");
    return true;
}

}  // namespace

int main() {
    if (!cases()) return 1;
    const size_t GiB = size_t(1) << 30;
    // a generous budget: pooled hierarchies are never released
    if (!simulate("roomy", 1, 3000, 2000.0, 512 * GiB, 64, SIZE_MAX, true)) return 1;
    // a budget that holds only a few large hierarchies: eviction and waiting
    if (!simulate("tight_budget", 2, 3000, 2000.0, 2 * GiB, 16, SIZE_MAX, false)) return 1;
    // device memory below the budget: allocations answer out-of-memory
    if (!simulate("device_oom", 3, 2000, 500.0, 64 * GiB, 32, GiB + GiB / 2, false)) return 1;
    // one slot per dimension: strictly serial per dimension
    if (!simulate("one_slot", 4, 500, 50.0, 64 * GiB, 1, SIZE_MAX, true)) return 1;
    return g_fail;
}
