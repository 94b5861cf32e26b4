// Solver core: the V-cycle driver of Algorithm 1 over groups of equal-size
// grids, default launch geometry, and helper kernels for hierarchy setup.
#include <algorithm>
#include <cstdlib>
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

int heuristic_zchunk(int dim, int n, int by, int halo, int target_blocks) {
    if (dim == 2) return 1;
    const int m = n - 2;
    const int TX = 64 - 2 * halo, TY = by - 2 * halo;
    const int cols = ((m + TX - 1) / TX) * ((m + TY - 1) / TY);
    const int chunks = std::max(1, (target_blocks + cols - 1) / cols);
    return std::max(2, (m + chunks - 1) / chunks);
}

Tiles default_tiles(int dim, int elem_bytes, int n, int smoother) {
    Tiles t;
    const int H = smoother == SM_RBGS ? 2 : 1;
    const int target = 2048;
    if (dim == 2) {
        const int by = n >= 257 ? 32 : (n >= 65 ? 16 : 8);
        t.smooth = t.smooth_zg = t.smooth_pro = t.smooth_nrm = {by, 1};
        t.restr = {by < 16 ? 16 : by, 1};
        t.norm = {by, 1};
        return t;
    }
    // two rows per thread: within the register limit of every precision
    const int by = n >= 129 ? 16 : 8;
    t.smooth = t.smooth_zg = t.smooth_pro = t.smooth_nrm = {by, heuristic_zchunk(3, n, by, H, target), 1,
                                                           by >= 16 ? 8 : 4};
    const int nc = (n - 1) / 2 + 1;
    const int rb = 16;
    // restriction tiles: 30 x ((rb-3)/2) coarse nodes per z-chunk of coarse planes
    {
        const int mc = nc - 2;
        const int cols = ((mc + 29) / 30) * ((mc + (rb - 3) / 2 - 1) / ((rb - 3) / 2));
        const int chunks = std::max(1, (target + cols - 1) / std::max(cols, 1));
        t.restr = {rb, std::max(1, (mc + chunks - 1) / chunks)};
    }
    t.norm = {by, heuristic_zchunk(3, n, by, 1, target)};
    (void)elem_bytes;
    return t;
}

template <typename T>
hipError_t launch_smooth(int dim, int sm, bool var, const GridDesc* d, int ninst, int n, int sel, int flags,
                         TileCfg cfg, hipStream_t s) {
    if (n < 5 || ninst <= 0) return hipErrorInvalidValue;
    if ((flags & SWEEP_NORM) && ninst != 1) return hipErrorInvalidValue;  // one partial row
    const dim3 grid(smooth_tiles(dim, sm, n, cfg), ninst);
    const hipError_t e = dim == 2 ? launch_smooth2d<T>(sm, var, d, sel, flags, cfg, grid, s)
                                  : launch_smooth3d<T>(sm, var, d, sel, flags, cfg, grid, s);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}
template hipError_t launch_smooth<double>(int, int, bool, const GridDesc*, int, int, int, int, TileCfg, hipStream_t);
template hipError_t launch_smooth<float>(int, int, bool, const GridDesc*, int, int, int, int, TileCfg, hipStream_t);
template hipError_t launch_smooth<half_t>(int, int, bool, const GridDesc*, int, int, int, int, TileCfg, hipStream_t);

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

int tail_first_level(int dim, int elem, const std::vector<int>& n, bool zero_top) {
    if (std::getenv("MG_NO_TAIL")) return -1;
    if (n.empty() || n.back() != 3) return -1;  // the tail ends in the exact 3-node solve
    const int tmax = tail_max_edge(dim, elem);
    for (int l = zero_top ? 0 : 1; l < (int)n.size(); ++l)
        if (n[(size_t)l] <= tmax && (int)n.size() - l <= kMaxTailLevels) return l;
    return -1;
}

// Coarsest level: exact solve of the single unknown (n = 3) or conjugate
// gradients (n > 3), from a zero iterate.
template <typename T>
hipError_t coarse_solve(const Problem& P, const Group& g, hipStream_t s) {
    if (g.n == 3) return launch_coarsest<T>(P.dim, P.var, g.d, g.ninst, s);
    return launch_cg<T>(P.dim, P.var, g.d, g.ninst, g.n, P.cg_iters > 0 ? P.cg_iters : 4 * (g.n - 1), s);
}

// The fused last pre-smoothing sweep + restriction applies to 3D Laplacian
// red-black levels in FP32 or binary16 storage whose tiles chose it.
template <typename T>
bool fused_restrict_ok(const Problem& P, int dim, const Tiles& t) {
    return sizeof(T) <= 4 && dim == 3 && !P.var && P.smoother == SM_RBGS && t.fused.zchunk > 0 &&
           std::getenv("MG_NO_FUSED_RESTRICT") == nullptr;
}

// The first two pre-smoothing sweeps from a zero iterate in one launch:
// Laplacian red-black levels in FP32 or binary16 storage whose tiles chose it.
template <typename T>
bool smooth2_ok(const Problem& P, int dim, const Tiles& t, bool zero) {
    return zero && sizeof(T) <= 4 && (dim == 2 || dim == 3) && !P.var && P.smoother == SM_RBGS && P.nu1 >= 2 &&
           t.smooth_zg2.zchunk > 0 && std::getenv("MG_NO_FUSED_SMOOTH2") == nullptr;
}
// 'sel' names the output buffer (1: u, 0: t; the input is the zero iterate).
template <typename T>
hipError_t launch_smooth2(int dim, const Group& g, const Tiles& t, int sel, hipStream_t s) {
    return dim == 2 ? launch_smooth2d_zg2<T>(g.d, g.ninst, g.n, sel, t.smooth_zg2, s)
                    : launch_smooth3d_zg2<T>(g.d, g.ninst, g.n, sel, t.smooth_zg2, s);
}
// The first two post-smoothing sweeps (correction fused into the first) in one
// launch: 2D Laplacian red-black levels in FP32 or binary16 storage whose
// tiles chose it.
template <typename T>
bool post2_ok(const Problem& P, int dim, const Tiles& t) {
    return sizeof(T) <= 4 && dim == 2 && !P.var && P.smoother == SM_RBGS && P.nu2 >= 2 &&
           t.smooth_pro2.zchunk > 0 && std::getenv("MG_NO_FUSED_POST2") == nullptr;
}

// Post-smoothing select bits: the symmetric red-black smoother relaxes black first.
inline int post_sel(const Problem& P, int cur) { return cur | (P.sym ? SEL_BLACK_FIRST : 0); }

// Algorithm 1 on level l with gamma recursive calls: kind 0 V (one call), 1 W
// (two), 2 F (an F-cycle then a V-cycle).  The zero guess precedes the first
// call only; later calls continue from the coarse iterate the previous call
// left.  Level by level (no coarse tail).
template <typename T>
hipError_t cycle_rec(const Problem& P, const std::vector<Group>& G, int l, int kind, bool zero,
                     const std::vector<Tiles>& tiles, hipStream_t s, Prof& prof, bool first_done = false) {
    const int L = (int)G.size();
    const int dim = P.dim;
    const Group& g = G[(size_t)l];
    if (l == L - 1) return coarse_solve<T>(P, g, s);
    int cur = first_done ? 1 : 0;
    int i0 = first_done ? 1 : 0;
    if (!first_done && smooth2_ok<T>(P, dim, tiles[(size_t)l], zero)) {
        // sweeps 1 and 2 from the zero iterate: the result lands in u
        MG_TRY(launch_smooth2<T>(dim, g, tiles[(size_t)l], 1, s));
        i0 = 2;
    }
    for (int i = i0; i < P.nu1; ++i) {
        const int flags = (i == 0 && zero) ? SWEEP_ZERO_GUESS : 0;
        const bool timed = l == 0 && flags == 0;
        if (timed) prof.begin();
        MG_TRY(launch_smooth<T>(dim, P.smoother, P.var, g.d, g.ninst, g.n, cur, flags, tiles[(size_t)l].sweep(flags),
                                s));
        if (timed) prof.end();
        cur ^= 1;
    }
    if (P.nu1 == 0 && zero) MG_TRY(launch_zero_u<T>(dim, g.d, g.ninst, g.n, s));
    MG_TRY(launch_restrict<T>(dim, P.var, g.d, g.ninst, g.n, cur, tiles[(size_t)l].restr, s));
    if (kind == 0) {
        MG_TRY(cycle_rec<T>(P, G, l + 1, 0, true, tiles, s, prof));
    } else if (kind == 1) {
        MG_TRY(cycle_rec<T>(P, G, l + 1, 1, true, tiles, s, prof));
        MG_TRY(cycle_rec<T>(P, G, l + 1, 1, false, tiles, s, prof));
    } else {
        MG_TRY(cycle_rec<T>(P, G, l + 1, 2, true, tiles, s, prof));
        MG_TRY(cycle_rec<T>(P, G, l + 1, 0, false, tiles, s, prof));
    }
    const bool fuse = P.nu2 > 0;
    if (!fuse) MG_TRY(launch_prolong<T>(dim, g.d, g.ninst, g.n, cur, s));
    for (int i = 0; i < P.nu2; ++i) {
        const int flags = (i == 0 && fuse) ? SWEEP_PROLONG : 0;
        const bool timed = l == 0 && flags == 0;
        if (timed) prof.begin();
        MG_TRY(launch_smooth<T>(dim, P.smoother, P.var, g.d, g.ninst, g.n, post_sel(P, cur), flags,
                                tiles[(size_t)l].sweep(flags), s));
        if (timed) prof.end();
        cur ^= 1;
    }
    if (cur == 1) MG_TRY(launch_copy_t_to_u<T>(dim, g.d, g.ninst, g.n, s));
    return hipSuccess;
}

template <typename T>
hipError_t vcycle(const Problem& P, const std::vector<Group>& G, bool zero_top, const std::vector<Tiles>& tiles,
                  hipStream_t s, hipEvent_t* prof_ev, int* prof_n, int prof_cap, const TailPlan* tail,
                  bool first_done) {
    const int L = (int)G.size();
    const int dim = P.dim;
    Prof prof{prof_ev, prof_n, prof_cap, s};
    // a first sweep that already ran needs a level-0 pre-smoothing sweep to have been
    if (first_done && (L < 2 || P.nu1 < 1 || zero_top)) return hipErrorInvalidValue;
    if (P.cycle != 0) return cycle_rec<T>(P, G, 0, P.cycle, zero_top, tiles, s, prof, first_done);
    const bool use_tail = tail && tail->first >= 0 && tail->first < L && tail->d;
    // levels [0, stop) run level by level; the rest is the tail (or the coarsest solve)
    const int stop = use_tail ? tail->first : L - 1;
    if (first_done && stop == 0) return hipErrorInvalidValue;
    if (stop == 0 && !use_tail) return coarse_solve<T>(P, G[0], s);
    std::vector<int> sel((size_t)L, 0);
    // descending leg: presmoothing, residual, restriction (Algorithm 1)
    for (int l = 0; l < stop; ++l) {
        const Group& g = G[(size_t)l];
        const bool zero = l == 0 ? zero_top : true;
        // the last sweep may carry the residual and restriction (a plain red-first sweep)
        const bool skip1 = l == 0 && first_done;
        // sweeps 1 and 2 from the zero iterate in one launch (result in u)
        const bool two = !skip1 && smooth2_ok<T>(P, dim, tiles[(size_t)l], zero);
        const bool fuse = fused_restrict_ok<T>(P, dim, tiles[(size_t)l]) && P.nu1 >= (two ? 3 : (zero ? 2 : 1));
        int cur = skip1 ? 1 : 0;
        int i0 = skip1 ? 1 : 0;
        // with the fused post-smoothing pair on this level the two sweeps land
        // in t, so that the pair (t -> u) leaves the iterate in u
        const bool post2 = two && P.nu1 == 2 && post2_ok<T>(P, dim, tiles[(size_t)l]);
        if (two) {
            MG_TRY(launch_smooth2<T>(dim, g, tiles[(size_t)l], post2 ? 0 : 1, s));
            i0 = 2;
            cur = post2 ? 1 : 0;
        }
        for (int i = i0; i < P.nu1; ++i) {
            const int flags = (i == 0 && zero) ? SWEEP_ZERO_GUESS : 0;
            if (fuse && i == P.nu1 - 1) {
                MG_TRY(launch_smooth_restrict3d<T>(g.d, g.ninst, g.n, cur, tiles[(size_t)l].fused, s));
                cur ^= 1;
                continue;
            }
            const bool timed = l == 0 && flags == 0;  // plain finest-level sweeps only
            if (timed) prof.begin();
            MG_TRY(launch_smooth<T>(dim, P.smoother, P.var, g.d, g.ninst, g.n, cur, flags,
                                    tiles[(size_t)l].sweep(flags), s));
            if (timed) prof.end();
            cur ^= 1;
        }
        if (P.nu1 == 0 && zero) MG_TRY(launch_zero_u<T>(dim, g.d, g.ninst, g.n, s));
        if (!fuse) MG_TRY(launch_restrict<T>(dim, P.var, g.d, g.ninst, g.n, cur, tiles[(size_t)l].restr, s));
        sel[(size_t)l] = cur;
    }
    if (use_tail) {
        // every level from 'stop' to the coarsest in one launch, from a zero guess
        MG_TRY(launch_tail<T>(dim, P.smoother, P.var, tail->d, tail->ninst, P.nu1, P.nu2, P.sym ? 1 : 0, s));
    } else {
        // coarsest grid from the zero guess
        MG_TRY(coarse_solve<T>(P, G[(size_t)L - 1], s));
    }
    // ascending leg: interpolation + correction, postsmoothing
    for (int l = stop - 1; l >= 0; --l) {
        const Group& g = G[(size_t)l];
        int cur = sel[(size_t)l];
        const bool fuse = P.nu2 > 0;  // the first post-sweep adds P uc while loading
        if (!fuse) MG_TRY(launch_prolong<T>(dim, g.d, g.ninst, g.n, cur, s));
        int i0 = 0;
        if (cur == 1 && post2_ok<T>(P, dim, tiles[(size_t)l])) {
            // post-sweeps 1 and 2 (correction in the first), t -> u
            MG_TRY(launch_smooth2d_pro2<T>(g.d, g.ninst, g.n, post_sel(P, cur), tiles[(size_t)l].smooth_pro2, s));
            cur = 0;
            i0 = 2;
        }
        for (int i = i0; i < P.nu2; ++i) {
            const int flags = (i == 0 && fuse) ? SWEEP_PROLONG : 0;
            const bool timed = l == 0 && flags == 0;
            if (timed) prof.begin();
            MG_TRY(launch_smooth<T>(dim, P.smoother, P.var, g.d, g.ninst, g.n, post_sel(P, cur), flags,
                                    tiles[(size_t)l].sweep(flags), s));
            if (timed) prof.end();
            cur ^= 1;
        }
        if (cur == 1) MG_TRY(launch_copy_t_to_u<T>(dim, g.d, g.ninst, g.n, s));
    }
    return hipSuccess;
}

template hipError_t vcycle<double>(const Problem&, const std::vector<Group>&, bool, const std::vector<Tiles>&,
                                   hipStream_t, hipEvent_t*, int*, int, const TailPlan*, bool);
template hipError_t vcycle<float>(const Problem&, const std::vector<Group>&, bool, const std::vector<Tiles>&,
                                  hipStream_t, hipEvent_t*, int*, int, const TailPlan*, bool);
template hipError_t vcycle<half_t>(const Problem&, const std::vector<Group>&, bool, const std::vector<Tiles>&,
                                   hipStream_t, hipEvent_t*, int*, int, const TailPlan*, bool);

}  // namespace mg
