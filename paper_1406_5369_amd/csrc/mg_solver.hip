// Solver core: the V-cycle driver of Algorithm 1 over groups of equal-size
// grids, default launch geometry, and helper kernels for hierarchy setup.
#include <algorithm>
#include <cstring>

#include "mg_solver.h"

namespace mg {

size_t npts(int dim, int n) { return dim == 2 ? (size_t)n * n : (size_t)n * n * n; }

int count_levels(int n) {
    int L = 1;
    while (n > 3) {
        n = (n - 1) / 2 + 1;
        ++L;
    }
    return L;
}

Tiles default_tiles(int dim, int elem_bytes) {
    Tiles t;
    if (dim == 2) {
        t.smooth = {32, 1};
        t.restr = {32, 1};
        t.norm = {32, 1};
    } else if (elem_bytes == 8) {
        t.smooth = {16, 128};
        t.restr = {16, 64};
        t.norm = {16, 128};
    } else {
        t.smooth = {16, 128};
        t.restr = {16, 64};
        t.norm = {16, 128};
    }
    return t;
}

namespace {

// Launch + optional event bracket (finest-level smoothing measurement).
struct Prof {
    hipEvent_t* ev;
    int* n;
    int cap;
    hipStream_t s;
    bool on() const { return ev && n && *n + 2 <= cap; }
    void begin() {
        if (on()) (void)hipEventRecord(ev[*n], s);
    }
    void end() {
        if (on()) {
            (void)hipEventRecord(ev[*n + 1], s);
            *n += 2;
        }
    }
};

}  // namespace

#define MG_TRY(x)                          \
    do {                                   \
        hipError_t e_ = (x);               \
        if (e_ != hipSuccess) return e_;   \
    } while (0)

template <typename T>
hipError_t vcycle(const Problem& P, const std::vector<Group>& G, bool zero_top, const Tiles& tiles, hipStream_t s,
                  hipEvent_t* prof_ev, int* prof_n, int prof_cap) {
    const int L = (int)G.size();
    const int dim = P.dim;
    Prof prof{prof_ev, prof_n, prof_cap, s};
    if (L == 1) return launch_coarsest<T>(dim, P.var, G[0].d, G[0].ninst, s);
    std::vector<int> sel((size_t)L, 0);
    // descending leg: presmoothing, residual, restriction (Algorithm 1)
    for (int l = 0; l + 1 < L; ++l) {
        const Group& g = G[(size_t)l];
        const bool zero = l == 0 ? zero_top : true;
        int cur = 0;
        for (int i = 0; i < P.nu1; ++i) {
            const int flags = (i == 0 && zero) ? SWEEP_ZERO_GUESS : 0;
            if (l == 0) prof.begin();
            MG_TRY(launch_smooth<T>(dim, P.smoother, P.var, g.d, g.ninst, g.n, cur, flags, tiles.smooth, s));
            if (l == 0) prof.end();
            cur ^= 1;
        }
        if (P.nu1 == 0 && zero) MG_TRY(launch_zero_u<T>(dim, g.d, g.ninst, g.n, s));
        MG_TRY(launch_restrict<T>(dim, P.var, g.d, g.ninst, g.n, cur, tiles.restr, s));
        sel[(size_t)l] = cur;
    }
    // coarsest grid: exact solve from the zero guess
    MG_TRY(launch_coarsest<T>(dim, P.var, G[(size_t)L - 1].d, G[(size_t)L - 1].ninst, s));
    // ascending leg: interpolation + correction, postsmoothing
    for (int l = L - 2; l >= 0; --l) {
        const Group& g = G[(size_t)l];
        int cur = sel[(size_t)l];
        const bool fuse = P.nu2 > 0 && dim == 2;  // 2D sweeps add P uc while loading
        if (!fuse) MG_TRY(launch_prolong<T>(dim, g.d, g.ninst, g.n, cur, s));
        for (int i = 0; i < P.nu2; ++i) {
            const int flags = (i == 0 && fuse) ? SWEEP_PROLONG : 0;
            if (l == 0) prof.begin();
            MG_TRY(launch_smooth<T>(dim, P.smoother, P.var, g.d, g.ninst, g.n, cur, flags, tiles.smooth, s));
            if (l == 0) prof.end();
            cur ^= 1;
        }
        if (cur == 1) MG_TRY(launch_copy_t_to_u<T>(dim, g.d, g.ninst, g.n, s));
    }
    return hipSuccess;
}

template hipError_t vcycle<double>(const Problem&, const std::vector<Group>&, bool, const Tiles&, hipStream_t,
                                   hipEvent_t*, int*, int);
template hipError_t vcycle<float>(const Problem&, const std::vector<Group>&, bool, const Tiles&, hipStream_t,
                                  hipEvent_t*, int*, int);

}  // namespace mg
