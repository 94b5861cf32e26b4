// Solver core: level hierarchies, the V-cycle driver (Algorithm 1), the
// solve loop with device-side stop test, FP64 iterative refinement around
// FP32 V-cycles, hipGraph capture and the tile autotuner.
#pragma once

#include <string>
#include <vector>

#include "../../include/mg.h"
#include "mg_internal.h"

struct mg_ctx;

namespace mg {

// Launch geometry of every kernel family of one hierarchy.
struct Tiles {
    TileCfg smooth{16, 128};      // plain sweep
    TileCfg smooth_zg{16, 128};   // sweep from a zero iterate (first presmoothing sweep on coarse grids)
    TileCfg smooth_pro{16, 128};  // sweep with the coarse-grid correction fused in (first postsmoothing sweep)
    TileCfg restr{16, 64};
    TileCfg norm{16, 128};
    // last pre-smoothing sweep fused with the residual and restriction (3D
    // Laplacian RBGS, FP32 / binary16): zchunk coarse planes per workgroup,
    // 0 = separate sweep and restriction (the autotuner's choice)
    TileCfg fused{16, 0};
    // FP64 finest level: the first pre-smoothing sweep that also sums r^2 of
    // its incoming iterate (an LDS tile geometry)
    TileCfg smooth_nrm{16, 128, 1, 8};
    // 3D Laplacian red-black, FP32 / binary16: the first two pre-smoothing
    // sweeps from a zero iterate in one launch (rows 12 or 16, zchunk planes
    // per workgroup; zchunk 0 = two separate sweeps, the autotuner's choice)
    TileCfg smooth_zg2{12, 0};
    // 2D Laplacian red-black, FP32 / binary16: the first two post-smoothing
    // sweeps (the coarse-grid correction fused into the first) in one launch
    // (zchunk rows per wavefront; 0 = separate sweeps, the autotuner's choice)
    TileCfg smooth_pro2{12, 0};
    const TileCfg& sweep(int flags) const {
        if (flags & SWEEP_NORM) return smooth_nrm;
        return (flags & SWEEP_ZERO_GUESS) ? smooth_zg : ((flags & SWEEP_PROLONG) ? smooth_pro : smooth);
    }
};

// Heuristic launch geometry for one level (used when autotuning is off and
// for levels too small to be worth timing): enough workgroups to cover the
// chip (z-chunks in 3D) and the smallest tile height on small grids.
Tiles default_tiles(int dim, int elem_bytes, int n, int smoother);
// Autotune the FP32 sweeps and restriction of one absolute level of a batch:
// 'count' instances of edge n, descriptors d (device).  Cached per process.
hipError_t tune_group(int dim, int smoother, const GridDesc* d, int count, int n, Tiles& t, hipStream_t s);
int heuristic_zchunk(int dim, int n, int by, int halo, int target_blocks);

// Device buffers of one instance's hierarchy in working precision T
// (sizeof(T) bytes per value).  Level 0 buffers may belong to the caller.
struct Levels {
    int dim = 0, nlev = 0, elem = 8;
    std::vector<int> n;           // n[0] finest
    std::vector<void*> u, t, f, k;  // per level; k empty when Laplacian
    std::vector<void*> fx;          // 3D with k: face coefficients of levels the sweeps run on (GridDesc::fx)
    std::vector<char> own_u, own_f; // level owns u / f
    bool own_k0 = false;            // level-0 coefficient allocated by the hierarchy
};

// A group of instances that share one level size: one launch processes all.
struct Group {
    int n = 0;
    int ninst = 0;
    GridDesc* d = nullptr;         // device descriptors [ninst]
    std::vector<GridDesc> h;       // host mirror
};

struct Problem {
    int dim, smoother, nu1, nu2;  // smoother: SM_RBGS or SM_JACOBI (the kernels' relaxations)
    double omega;
    bool var;
    bool sym = false;   // symmetric red-black: the post-smoothing sweeps relax black first
    int cycle = 0;      // 0 V, 1 W, 2 F (Algorithm 1 with one / two recursive calls; F: F then V)
    int cg_iters = 0;   // conjugate-gradient steps on a coarsest level with n > 3 (0: 4 (n - 1))
};

// Coarse levels of a V-cycle run by the single-workgroup tail kernel:
// groups[first..L-1], one TailDesc per instance (first = -1: no tail).
struct TailPlan {
    int first = -1;
    int ninst = 0;
    TailDesc* d = nullptr;  // device [ninst]
};

// First level of a hierarchy (edges n[0] > n[1] > ... > 3) that the tail kernel
// takes, or -1: the largest level with an edge up to tail_max_edge, not the
// top level unless its iterate starts at zero.  MG_NO_TAIL disables the tail.
int tail_first_level(int dim, int elem, const std::vector<int>& n, bool zero_top);

// V-cycle over groups[0..L-1] (groups[l] holds every instance's level l);
// zero_top: the iterate at level 0 is known to be zero.  Works in precision T.
// first_done: level 0's first pre-smoothing sweep has already run (its result
// is in the ping-pong partner t; the cycle continues from the second sweep).
template <typename T>
hipError_t vcycle(const Problem& P, const std::vector<Group>& groups, bool zero_top, const std::vector<Tiles>& tiles,
                  hipStream_t s, hipEvent_t* prof_ev, int* prof_n, int prof_cap, const TailPlan* tail = nullptr,
                  bool first_done = false);

size_t npts(int dim, int n);
int count_levels(int n);

// Batched / served contexts share the opaque mg_ctx handle type.
bool is_batch_handle(const mg_ctx* c);
void destroy_batch_handle(mg_ctx* c);

}  // namespace mg

// The opaque context of the C ABI.
struct mg_ctx {
    mg_params p;
    int device = 0;
    hipStream_t stream = nullptr;
    mg::Problem prob{};
    int nlev = 0;
    std::vector<int> n;
    std::vector<mg::Tiles> tl64, tl32;  // per level launch geometry of each hierarchy
    mg::Tiles top;                      // finest-level FP64 norm / refinement kernels
    bool autotune = true;

    // FP64 hierarchy (precision FP64): level 0 u/f are the caller's.
    mg::Levels L64;
    std::vector<mg::Group> G64;
    mg::TailPlan tail64;
    // FP32 hierarchy (precision FP32_IR): all levels owned; level-0 u = e, f = r32.
    mg::Levels L32;
    std::vector<mg::Group> G32;
    mg::TailPlan tail32;
    // FP32_IR and FP16_IR share these members: L32 / G32 / tail32 / tl32 hold
    // the hierarchy of the refinement's cycles, in FP32 or binary16 (L32.elem)
    // FP64 refinement state
    double* d_scl = nullptr;   // FP16_IR: {scale of the correction, largest |r| of the last pass}
    double* d_pmax = nullptr;  // FP16_IR: partial maxima of |r| (pstride)
    mg::IRDesc* d_ir = nullptr;
    mg::IRDesc h_ir{};
    double* u64_scratch = nullptr;
    double* k64 = nullptr;  // private copy of the FP64 nodal coefficient (var-coef)

    // solve control (one instance)
    double* d_partial = nullptr;
    int pstride = 0;
    // FP64 solves: the residual norm of each cycle's result is summed by the
    // next cycle's first pre-smoothing sweep (one partial per workgroup of it)
    bool nrm_fused = false;
    double* d_spart = nullptr;
    int spart_cap = 0;
    double* d_norm = nullptr;   // [1]
    double* d_norm0 = nullptr;  // [1]
    double* d_hist = nullptr;
    int hist_cap = 0;
    double* h_pin = nullptr;  // pinned host staging

    mg::GridDesc* d_top = nullptr;  // FP64 view of the finest level (residual norms)
    mg::GridDesc h_top{};
    int* d_ctrl = nullptr;            // done, steps, status

    const void* bound_u = nullptr;
    const void* bound_f = nullptr;

    // captured chunks of solve steps, by step count, starting parity of the
    // refinement ping-pong, tolerance and step limit
    struct ChunkGraph {
        int steps, par, max_cycles;
        double tol;
        hipGraphExec_t exec;
    };
    bool use_graphs = true;
    hipStream_t cap_stream = nullptr;
    std::vector<ChunkGraph> graphs;

    // cell-centred Neumann grid (bc MG_BC_NEUMANN_CC): levels n, n/2, ..., 1 cells
    // per axis; level 0's iterate is the caller's, its right-hand side the
    // context's mean-zero copy ccfh
    bool cc = false;
    std::vector<int> ccn;
    std::vector<double*> ccu, cct, ccf;
    double* ccfh = nullptr;
    double* cc_work = nullptr;  // fixed-order sums (row and plane sums)
    double* cc_mean = nullptr;  // [1]

    // complex diffusion (mg_cdiff_setup): its level hierarchy
    struct CDState* cd = nullptr;

    // constant stencil (op MG_OP_CONST_STENCIL): the stencil and levels n, ...,
    // 3 with their iterate (level 0: the caller's), Jacobi partner and
    // right-hand side (level 0: the caller's)
    bool st = false;
    double st_coef[7] = {0, 0, 0, 0, 0, 0, 0};
    std::vector<int> stn;
    std::vector<double*> stu, stt, stf;

    // measurement
    // measurement hooks: event pairs of the current solve, tagged with their
    // refinement step and kernel (0 finest plain sweeps, 1 finest refinement /
    // norm pass); only steps the solve really ran are added to the totals
    bool prof_on = false;
    std::vector<hipEvent_t> prof_ev;
    int prof_n = 0;
    std::vector<int> prof_step, prof_kind;  // per event pair
    int prof_launches[2] = {0, 0};
    double prof_ms[2] = {0.0, 0.0};
};
