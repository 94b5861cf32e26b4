// Admission and retirement policy of the serving loop (host code only).
//
// Requests wait in arrival order.  The head of the queue is admitted when its
// dimension has a free instance slot and its hierarchy fits the device-memory
// budget: a pooled hierarchy of the same edge is reused; otherwise pooled
// hierarchies of other edges are released (in key order) until a new one fits
// the budget, and more of them while the device reports out-of-memory; if it
// still does not fit, the head waits for running requests to retire.
// The head is never overtaken, so no request starves while others complete.
// A retired request's hierarchy goes back to the pool of its edge and keeps
// counting against the budget until it is reused or released.
//
// The policy is generic over the hierarchy handle H and a backend B that owns
// device memory:
//   size_t B::bytes(int dim, int n)        bytes a new hierarchy of that edge takes
//   size_t B::bytes_of(H h)                bytes held by an existing one
//   int    B::alloc(int dim, int n, H* h)  0 ok, 1 out of memory (wait), < 0 error
//   void   B::release(H h)                 free a pooled hierarchy
#pragma once

#include <cstddef>
#include <deque>
#include <map>
#include <utility>
#include <vector>

namespace mg {

template <class H>
struct Sched {
    size_t budget = 0;  // bytes that admitted and pooled hierarchies may hold
    int slots = 0;      // concurrent requests per dimension (2D, 3D)
    size_t used = 0;    // bytes held now (active + pooled)
    int active = 0;
    std::deque<long long> queue;  // ids in arrival order
    std::vector<char> slot_used[2];
    std::map<std::pair<int, int>, std::vector<H>> pool;  // (dim, n) -> free hierarchies

    void init(size_t budget_bytes, int slots_per_dim) {
        budget = budget_bytes;
        slots = slots_per_dim;
        for (auto& v : slot_used) v.assign((size_t)slots_per_dim, 0);
    }

    void submit(long long id) { queue.push_back(id); }

    int free_slot(int dim) const {
        const std::vector<char>& v = slot_used[dim - 2];
        for (int i = 0; i < (int)v.size(); ++i)
            if (!v[(size_t)i]) return i;
        return -1;
    }

    // Try to admit the head of the queue, whose edge is (dim, n).  Returns 1 and
    // fills slot / h when admitted (the head is popped), 0 when the head must
    // wait, or the backend's negative error code.
    template <class B>
    int admit_head(B& b, int dim, int n, int* slot_out, H* h_out) {
        if (queue.empty()) return 0;
        const int slot = free_slot(dim);
        if (slot < 0) return 0;
        H h{};
        auto& same = pool[{dim, n}];
        if (!same.empty()) {
            h = same.back();
            same.pop_back();
        } else {
            const size_t need = b.bytes(dim, n);
            for (auto it = pool.begin(); used + need > budget && it != pool.end(); ++it)
                while (!it->second.empty() && used + need > budget) {
                    H v = it->second.back();
                    it->second.pop_back();
                    used -= b.bytes_of(v);
                    b.release(v);
                }
            if (used + need > budget) return 0;
            int r = b.alloc(dim, n, &h);
            while (r == 1) {  // device memory is short: give pooled hierarchies back one at a time
                bool freed = false;
                for (auto it = pool.begin(); it != pool.end() && !freed; ++it)
                    if (!it->second.empty()) {
                        H v = it->second.back();
                        it->second.pop_back();
                        used -= b.bytes_of(v);
                        b.release(v);
                        freed = true;
                    }
                if (!freed) return 0;  // wait for running requests to retire
                r = b.alloc(dim, n, &h);
            }
            if (r < 0) return r;
            used += b.bytes_of(h);
        }
        slot_used[dim - 2][(size_t)slot] = 1;
        ++active;
        queue.pop_front();
        *slot_out = slot;
        *h_out = h;
        return 1;
    }

    // A request in (dim, slot) with hierarchy h of edge n has completed.
    void retire(int dim, int slot, int n, H h) {
        slot_used[dim - 2][(size_t)slot] = 0;
        pool[{dim, n}].push_back(h);
        --active;
    }

    // Release every pooled hierarchy (at shutdown).
    template <class B>
    void drain_pool(B& b) {
        for (auto& kv : pool)
            for (H v : kv.second) {
                used -= b.bytes_of(v);
                b.release(v);
            }
        pool.clear();
    }
};

}  // namespace mg
