// Internal declarations shared by the HIP kernels and the solver core.
// (Not part of the public C ABI; see include/mg.h for that.)
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace mg {

// binary16 storage cell of the half-precision hierarchy (arithmetic in float)
typedef _Float16 half_t;

// Largest accepted grid edges: every node index of a grid (and of each level)
// then fits in 32 bits (32769^2 and 1025^3 are both below 2^31).
constexpr int kMaxEdge2D = 32769, kMaxEdge3D = 1025;

// n = 2^L + 1 nodes per axis, L >= 1, within the size limit of its dimension.
inline bool valid_edge(int dim, int n) {
    return (dim == 2 || dim == 3) && n >= 3 && ((n - 1) & (n - 2)) == 0 && n <= (dim == 2 ? kMaxEdge2D : kMaxEdge3D);
}

// Largest tile height (rows of a 64-wide tile) of a kernel family: the 3D
// marching kernels keep three planes of their rows in registers, and with
// FP64 words or a coefficient field more than four rows per thread would not
// fit the 256 architectural VGPRs.  family: 0 smoothing, 1 residual +
// restriction, 2 FP64 norm / refinement pass; wv: wavefronts per workgroup.
inline int max_tile_rows(int dim, int elem, bool var, int family, int wv = 4) {
    if (dim == 2 || family == 1) return 32;
    if (wv == 1) {  // 3D sweep with one wavefront per tile: the thread holds every row
        if (family != 0) return 0;
        return elem <= 4 && !var ? 12 : (elem == 8 && var ? 0 : 8);
    }
    // 3D sweeps: FP64 with a coefficient field keeps six ring values per row
    // (iterate, coefficient and four face rings) in 8-byte registers
    const int rows_per_thread =
        family == 0 ? (elem == 8 && var ? 2 : (elem == 8 || var ? 4 : 8)) : (var ? 4 : 8);
    return rows_per_thread * wv < 32 ? rows_per_thread * wv : 32;
}

enum Smoother { SM_RBGS = 0, SM_JACOBI = 1 };

// Kernel flags for the smoothing sweep.
enum SweepFlags {
    SWEEP_ZERO_GUESS = 1,  // the incoming iterate is identically zero: read nothing
    SWEEP_PROLONG = 2,     // incoming iterate is u + P uc (coarse-grid correction fused into the load)
    SWEEP_NORM = 4,        // FP64 Laplacian / coefficient-field sweeps of an LDS tile geometry: also sum
                           // r^2 = (f - A u)^2 of the incoming iterate over the tile's output nodes
                           // into npart[blockIdx.x] (one partial per workgroup)
};

// One grid at one level, as the kernels see it.  All pointers are device
// pointers to dense node arrays (n^dim values, x fastest, boundary included).
// Sweeps ping-pong between u and t; 'sel' kernel arguments name the input
// buffer (0: u, 1: t).  The coarse iterate of a V-cycle always ends in u.
struct GridDesc {
    void* u;          // iterate
    void* t;          // ping-pong partner of u (same shape)
    const void* f;    // right-hand side
    const void* k;    // nodal diffusion coefficient, or null for the Laplacian
    const void* fx;   // 3D with k: face coefficients in the arithmetic type, three arrays of n^3
                      // values (+x, +y, +z face of every node; 1 where the face leaves the grid),
                      // read by the LDS sweeps; null otherwise
    void* uc;         // next coarser level's u (prolongation source), or null
    void* fc;         // next coarser level's f (restriction target), or null
    const int* done;  // per-instance stop flag (non-zero: skip), or null
    int n;            // nodes per axis
    int inst;         // instance number (index of this grid's norm partial row)
    double c;         // 1/h^2
    double wd;        // omega*h^2/(2d)
    double omega;     // smoother weight
    double* npart;    // SWEEP_NORM: per-workgroup partial sums of r^2 (as many as the launch has
                      // workgroups in x), or null
};

// FP64 refinement pass of one grid: u_out = u_in + e (inner nodes),
// r = f - A u_out in FP64, r32 = (float) r, per-block partial sums of r^2.
// Half-precision form: e and r are binary16 cells scaled by powers of two,
// u_out = u_in + e / scl[0] and r16 = half(float(s) * float(r)) with s the
// scale of scl[1] (the largest |r| of the previous pass); the pass also writes
// per-block partial maxima of |r| to pmax.
struct IRDesc {
    double* u[2];     // ping-pong FP64 iterate; kernel argument 'sel' names the input
    const void* e;    // correction, float (or binary16), zero boundary
    const double* f;  // FP64 right-hand side
    const double* k;  // FP64 nodal coefficient or null
    void* r;          // residual out, float (or binary16) (boundary left untouched, zero)
    const int* done;  // stop flag or null
    const int* par;   // per-instance ping-pong parity (overrides 'sel') or null
    int n;
    int inst;
    double c;
    const double* scl = nullptr;  // half-precision form: {scale of e, largest |r| of the previous pass}
    double* pmax = nullptr;       // half-precision form: partial maxima of |r|, same layout as the sums
};

// Coarse tail of a V-cycle for one instance: its levels from the tail's finest
// (lv[0], edge at most tail_max_edge) down to n = 3, run by one workgroup.
constexpr int kMaxTailLevels = 6;
struct TailDesc {
    GridDesc lv[kMaxTailLevels];
    int nlev;
};

// Launch geometry of one kernel family (picked by the autotuner).
struct TileCfg {
    int by;      // LDS box rows (2D) / rows of the x-y box (3D): 8, 16 or 32
    int zchunk;  // 3D: output planes per workgroup; 2D pass with xp 2: rows per wavefront
    int pd = 1;  // 3D smoothing: planes of old u prefetched ahead (1 or 2)
    int wv = 4;  // 3D smoothing: wavefronts per workgroup (1, 4 or 8); a thread holds by/wv rows
    int order = 0;  // smoothing: block-to-tile order, 0 XCD bands (see xcd_tile), 1 linear
    int xp = 1;     // norm / refinement pass (Laplacian): nodes per lane along x (1 or 2)
};

// Smoothing kernels take the input-buffer select, the block order and the
// colour order in one argument: bit 0 the select, bit 1 linear block order,
// bit 2 black first (red-black Gauss-Seidel: the colour (i+j[+k]) mod 2 = 1
// is relaxed before colour 0, the post-smoothing sweeps of the symmetric
// red-black smoother).  Callers pass bits 0 and 2 in 'sel'.
constexpr int SEL_BLACK_FIRST = 4;
inline int sweep_arg(int sel, const TileCfg& c) { return (sel & (1 | SEL_BLACK_FIRST)) | (c.order ? 2 : 0); }

// Number of workgroups in x for a level of n nodes per axis (one instance).
int smooth_tiles(int dim, int sm, int n, TileCfg cfg);
int restrict_tiles(int dim, int nf, TileCfg cfg);
int smooth_restrict_tiles(int nf, TileCfg cfg);
int smooth2_tiles(int n, TileCfg cfg);
int norm_tiles(int dim, int n, TileCfg cfg);

// Kernel launchers.  'ninst' grids with equal n are processed by one launch
// (blockIdx.y selects the descriptor).  'T' is double or float.
template <typename T>
hipError_t launch_smooth(int dim, int sm, bool var, const GridDesc* d, int ninst, int n, int sel, int flags,
                         TileCfg cfg, hipStream_t s);
// Per-dimension sweep launchers behind launch_smooth (grid already sized).
template <typename T>
hipError_t launch_smooth2d(int sm, bool var, const GridDesc* d, int sel, int flags, TileCfg cfg, dim3 grid,
                           hipStream_t s);
template <typename T>
hipError_t launch_smooth3d(int sm, bool var, const GridDesc* d, int sel, int flags, TileCfg cfg, dim3 grid,
                           hipStream_t s);
// 3D Laplacian, FP32 or binary16 storage: the first two red-first RBGS
// pre-smoothing sweeps from a zero iterate in one launch, the second sweep's
// result written to the output buffer of select 'sel' (1: u); cfg.by 12 or 16
// rows, cfg.zchunk planes per workgroup, cfg.order the block order.
template <typename T>
hipError_t launch_smooth3d_zg2(const GridDesc* d, int ninst, int n, int sel, TileCfg cfg, hipStream_t s);
// The same in 2D: cfg.zchunk rows per wavefront (128-node strips, four chunks
// of a strip per workgroup), cfg.order the block order.
template <typename T>
hipError_t launch_smooth2d_zg2(const GridDesc* d, int ninst, int n, int sel, TileCfg cfg, hipStream_t s);
int smooth2d_zg2_tiles(int n, int ychunk);
// 2D Laplacian, FP32 or binary16 storage: the first two red-black
// post-smoothing sweeps of input 'sel' in one launch, the coarse-grid
// correction from uc added as rows enter (sel bit 2: black first), the result
// written to the ping-pong partner of the input; cfg.zchunk rows per
// wavefront, cfg.order the block order.
template <typename T>
hipError_t launch_smooth2d_pro2(const GridDesc* d, int ninst, int n, int sel, TileCfg cfg, hipStream_t s);
int smooth2d_pro2_tiles(int n, int ychunk);
// 3D Laplacian, FP32 or binary16 storage: the last red-first RBGS pre-smoothing
// sweep of input 'sel' fused with the residual of its result and full
// weighting into fc (cfg.by 16 rows, cfg.zchunk coarse planes per workgroup,
// cfg.order the block order).
template <typename T>
hipError_t launch_smooth_restrict3d(const GridDesc* d, int ninst, int nf, int sel, TileCfg cfg, hipStream_t s);
template <typename T>
hipError_t launch_restrict(int dim, bool var, const GridDesc* d, int ninst, int nf, int sel, TileCfg cfg,
                           hipStream_t s);
template <typename T>
hipError_t launch_prolong(int dim, const GridDesc* d, int ninst, int nf, int sel, hipStream_t s);
// Largest tail edge for a dimension and word size (levels at or below it can
// run in the single-workgroup tail kernel).
int tail_max_edge(int dim, int elem);
template <typename T>
// post_first: colour relaxed first in the post-smoothing sweeps (0 red, 1 black).
hipError_t launch_tail(int dim, int sm, bool var, const TailDesc* d, int ninst, int nu1, int nu2, int post_first,
                       hipStream_t s);
// Conjugate gradients on a coarsest level of edge n (3 <= n <= tail_max_edge),
// 'iters' steps from u = 0, one workgroup per instance.
template <typename T>
hipError_t launch_cg(int dim, bool var, const GridDesc* d, int ninst, int n, int iters, hipStream_t s);
template <typename T>
hipError_t launch_coarsest(int dim, bool var, const GridDesc* d, int ninst, hipStream_t s);
template <typename T>
hipError_t launch_copy_t_to_u(int dim, const GridDesc* d, int ninst, int n, hipStream_t s);
template <typename T>
hipError_t launch_zero_u(int dim, const GridDesc* d, int ninst, int n, hipStream_t s);

// FP64 residual norm partials: partial[inst * pstride + block] = sum r^2 over the block.
hipError_t launch_norm(int dim, bool var, const GridDesc* d, int ninst, int n, int sel, double* partial,
                       int pstride, TileCfg cfg, hipStream_t s);
// FP64 refinement pass (see IRDesc); same partial layout as launch_norm.
// flags & IR_NO_UPDATE: u is not changed (e not read, u_out not written).
enum IRFlags { IR_NO_UPDATE = 1 };
hipError_t launch_ir_update(int dim, bool var, const IRDesc* d, int ninst, int n, int sel, int flags,
                            double* partial, int pstride, TileCfg cfg, hipStream_t s);
// Half-precision form of the pass (binary16 e and r, Laplacian, two nodes per
// lane: cfg.xp must be 2); also writes partial maxima of |r| to d->pmax.
hipError_t launch_ir_update_f16(int dim, const IRDesc* d, int ninst, int n, int sel, int flags, double* partial,
                                int pstride, TileCfg cfg, hipStream_t s);
// After a half-precision pass: norm = sqrt(sum of the partials) as
// launch_norm_finalize; unless *done: scl[0] = fp16 scale of scl[1] (the
// scale that pass wrote r with), scl[1] = max of the partial maxima.
hipError_t launch_norm_finalize_f16(const double* partial, const double* pmax, int nparts, double* norm, double* scl,
                                    const int* done, hipStream_t s);
// norm[inst] = sqrt(sum of partial[inst*pstride + 0 .. nparts-1]) in a fixed order; for
// each of 'ninst' rows starting at row 'row0'.
hipError_t launch_norm_finalize(const double* partial, int pstride, int nparts, int row0, int ninst,
                                double* norm, hipStream_t s);

// Device-side solve control, one entry per instance i in [0, ninst):
//   solve_init: norm0[i] = norm[i], hist[i*hstride] = norm[i], steps[i] = 0,
//               status[i] = 1 (running) / 0 (zero residual) / -5, done[i] set unless running.
//   stop_test:  for running instances: steps[i]++, hist[i*hstride+steps] = norm[i],
//               status 0 when norm <= tol*norm0, -5 on NaN/Inf/growth > 1e6,
//               2 when steps reaches max_steps; done[i] = 1 once status != 1.
hipError_t launch_solve_init(const double* norm, double* norm0, int* done, int* steps, int* status, double* hist,
                             int hstride, int ninst, hipStream_t s);
hipError_t launch_stop_test(const double* norm, const double* norm0, int* done, int* steps, int* status, double* hist,
                            int hstride, double tol, int max_steps, int ninst, hipStream_t s, int* par = nullptr);
// Batched variants over an explicit list of instance rows.
//   finalize_rows: norm[r] = sqrt(sum of partial[r*pstride + 0 .. nparts[r]-1]) for r in rows
//   solve_init_rows: as launch_solve_init for the listed rows (par[r] = 0 when par is given)
hipError_t launch_norm_finalize_rows(const double* partial, int pstride, const int* nparts, const int* rows, int nrows,
                                     double* norm, hipStream_t s);
// arr[rows[j]] = v for j < nrows.
hipError_t launch_set_rows(int* arr, int v, const int* rows, int nrows, hipStream_t s);
hipError_t launch_solve_init_rows(const double* norm, double* norm0, int* done, int* steps, int* status, int* par,
                                  const int* rows, int nrows, hipStream_t s);

// Face coefficients of a 3D level (GridDesc::fx) from its nodal k:
// fx[p] = kface(k_p, k_{p+x}), fx[N+p] = kface(k_p, k_{p+y}), fx[2N+p] = kface(k_p, k_{p+z}).
template <typename T>
hipError_t launch_faces3d(const T* k, T* fx, int n, hipStream_t s);
// Coarse coefficient by injection: dst(I) = (TD) src(2I) over every coarse node,
// nf = 2*nc - 1 nodes per axis on the fine side.
template <typename TS, typename TD>
hipError_t launch_inject(int dim, int nf, const TS* src, int nc, TD* dst, hipStream_t s);
// dst[q] = (TD) src[q] for q < total.
template <typename TS, typename TD>
hipError_t launch_convert(size_t total, const TS* src, TD* dst, hipStream_t s);
hipError_t launch_fill_int(int* p, int v, int count, hipStream_t s);

// Plain device copy of 'bytes' bytes (bandwidth calibration kernel).
hipError_t launch_copy_bytes(void* dst, const void* src, size_t bytes, hipStream_t s);

}  // namespace mg
