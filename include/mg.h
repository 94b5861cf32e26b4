/*
 * mg.h -- C ABI of the MI355X geometric multigrid library (libmg.so).
 *
 * The library solves the node-based finite-difference Poisson problem
 * -Laplace(u) = f on the unit square / cube with zero Dirichlet boundary
 * (Koestler et al., arXiv:1406.5369, Section 2.1 Eq. (1) and Section 2.2),
 * and the variable-coefficient problem -div(k grad u) = f in flux form with
 * harmonic-mean face coefficients, by the recursive multigrid V-cycle of
 * Algorithm 1 (Section 2.3): omega-Jacobi or red-black Gauss-Seidel smoothing,
 * full-weighting restriction, bi-/trilinear interpolation and correction, and
 * an exact solve on the coarsest 3 x 3 (x 3) grid.  The solve loop follows the
 * Layer-4 Application function (Section 2.4): L2 residual before and after
 * every cycle.
 *
 * Conventions shared by every entry point:
 *   - A grid has n = 2^L + 1 nodes per axis (L >= 1) including the boundary,
 *     spacing h = 1/(n-1), and is stored as one dense array of n^dim values,
 *     x fastest: idx = (k*n + j)*n + i (3D), j*n + i (2D).
 *   - Array arguments are DEVICE pointers (HIP global memory) unless stated
 *     otherwise; the caller owns them.  Boundary entries of u must be zero;
 *     the library reads them as the Dirichlet value and never writes them.
 *     Boundary entries of f are ignored.
 *   - 'stream' is a hipStream_t passed as void*; all work is enqueued on it.
 *     Entry points that return host scalars synchronise that stream.
 *   - Return value: MG_OK (0) on success, > 0 for a non-fatal outcome
 *     (MG_ENOTCONV: u is valid but the tolerance was not reached), < 0 for an
 *     error.  On MG_EINVAL / MG_ENOTSUP nothing was enqueued and u is untouched.
 *   - A context is not thread-safe and is bound to one device (the current
 *     device at mg_setup) and one stream.
 */
#ifndef MG_H
#define MG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mg_ctx mg_ctx;

enum mg_status {
    MG_OK = 0,
    MG_ENOTCONV = 1,     /* max_cycles reached before the tolerance; u valid */
    MG_EINVAL = -1,      /* bad argument (size not 2^L+1, null pointer, ...) */
    MG_ENOTSUP = -2,     /* valid but unsupported combination */
    MG_ENOMEM = -3,      /* device allocation failed or budget exceeded */
    MG_EDEVICE = -4,     /* a HIP runtime call failed */
    MG_EDIVERGED = -5,   /* residual became NaN/Inf or grew by more than 1e6 */
    MG_EBUSY = -6        /* server: no slot or budget left for this request now */
};

enum mg_operator {
    MG_OP_LAPLACE = 0,        /* constant 5-point (2D) / 7-point (3D) stencil, Section 2.2 */
    MG_OP_CONST_STENCIL = 1,  /* a constant stencil of the caller's (Section 2.2 declares the discretisation
                                 as a stencil with constant entries): (A u)_p = (1/h^2)(s0 u_p + sW u_W +
                                 sE u_E + sS u_S + sN u_N [+ sB u_B + sT u_T]), the same stencil with each
                                 level's h (re-discretisation; consistent for a second-order operator,
                                 entries summing to zero, e.g. anisotropic diffusion); smoothing
                                 u + omega h^2 / s0 (f - A u).  MG_PREC_FP64 and coarse_n 0 or 3 only
                                 (MG_ENOTSUP otherwise); plain one-node-per-thread kernels, level by level */
    MG_OP_VARCOEF_NODAL = 2   /* -div(k grad u): nodal k, face k = 2 k_p k_q / (k_p + k_q) */
};
enum mg_bc {
    MG_BC_DIRICHLET_ZERO = 0,  /* node-based grid, n = 2^L + 1 nodes per axis, zero boundary values */
    MG_BC_NEUMANN_CC = 1       /* cell-centred grid (Table 1), n = 2^L cells per axis (L >= 1; at most
                                  8192 in 2D, 512 in 3D), h = 1/n, homogeneous Neumann boundary (zero
                                  flux: a neighbour outside the domain takes the cell's own value);
                                  arrays hold n^dim cell values, no boundary entries.  Restriction
                                  averages the 2^d children, interpolation is constant, the coarsest
                                  level is one cell (zero correction).  The operator is singular:
                                  mg_solve projects f onto mean zero (a context copy; the residual
                                  history is that of the projected f) and keeps u at mean zero after
                                  every cycle, sums in a fixed order.  MG_OP_LAPLACE, MG_PREC_FP64,
                                  RBGS or Jacobi smoothing, coarse_n 0 (MG_ENOTSUP otherwise). */
};
enum mg_smoother {
    MG_SMOOTH_RBGS = 0,     /* red-black Gauss-Seidel, red ((i+j[+k]) even) first, Section 2.4 */
    MG_SMOOTH_WJACOBI = 1,  /* weighted Jacobi, Section 2.3; omega 0.8 in Table 2 */
    MG_SMOOTH_RBGS_SYM = 2  /* symmetric red-black Gauss-Seidel (Table 1's red-black variants): red first
                               before the coarse-grid correction, black first after it */
};
enum mg_cycle {
    MG_CYCLE_V = 0,  /* Algorithm 1: one recursive call per level */
    MG_CYCLE_W = 1,  /* two recursive calls per level (the second from the first's coarse iterate) */
    MG_CYCLE_F = 2   /* an F-cycle call followed by a V-cycle call per level */
};
enum mg_precision {
    MG_PREC_FP64 = 0,     /* every step in FP64 */
    MG_PREC_FP32_IR = 1,  /* FP32 V-cycles on the correction equation inside FP64 iterative refinement */
    MG_PREC_FP16_IR = 2   /* the same with every V-cycle field stored as IEEE binary16 and computed in
                             FP32 (Table 1's data-type choice below single precision): each refinement
                             step hands the cycle its FP64 residual scaled by a power of two s, chosen
                             so that 8 <= s * max|r| < 16 with max|r| taken from the previous step's
                             residual (the first step measures its own; s is kept within 2^-126 ..
                             2^127), and adds the correction divided by s.  MG_OP_LAPLACE only (MG_ENOTSUP otherwise).  An overflow
                             of binary16 shows as MG_EDIVERGED. */
};

typedef struct mg_params {
    int dim;         /* 2 or 3 (unit square / unit cube, Table 1) */
    int n;           /* nodes per axis incl. boundary, 2^L + 1, L >= 1; at most 32769 in 2D
                        and 1025 in 3D, so every node index fits in 32 bits */
    int op;          /* enum mg_operator */
    const double* k; /* MG_OP_VARCOEF_NODAL: device pointer to n^dim positive FP64 nodal
                        coefficients, copied during mg_setup; otherwise ignored */
    int bc;          /* enum mg_bc (only MG_BC_DIRICHLET_ZERO) */
    int smoother;    /* enum mg_smoother */
    double omega;    /* relaxation weight; <= 0 selects the paper's value (1.0 RBGS, 0.8 Jacobi) */
    int nu1, nu2;    /* pre- and post-smoothing sweeps (paper: 2, 2); 0..16 */
    int precision;   /* enum mg_precision */
    int cycle;       /* enum mg_cycle (0: the V-cycle of Algorithm 1) */
    int coarse_n;    /* edge of the coarsest level, 2^c + 1 with 3 <= coarse_n <= n (0 or 3: the single
                        unknown of the 3-node grid, solved exactly); larger: conjugate gradients there
                        (Algorithm 1: "direct solver or CG"), from a zero iterate, with inner products
                        in FP64 (each x-row summed in order, then the rows); at most 33 (2D) / 9 (3D)
                        with MG_PREC_FP64, 65 / 17 otherwise (MG_ENOTSUP beyond) */
    int cg_iters;    /* CG steps on a coarsest level with coarse_n > 3 (0: 4 (coarse_n - 1)); fewer only
                        if the residual or p^T A p becomes zero */
    const double* stencil; /* MG_OP_CONST_STENCIL: HOST pointer to 2*dim + 1 finite coefficients, centre
                        first (> 0), then -x, +x, -y, +y[, -z, +z]; copied during mg_setup; otherwise
                        ignored */
    double h;        /* grid spacing: 0 selects the unit domain's (1/(n-1) on node grids, 1/n on
                        cell-centred grids); any other positive value must equal it (MG_ENOTSUP:
                        other domain sizes are not built), negative or non-finite: MG_EINVAL */
} mg_params;

/* Build the level hierarchy n, (n-1)/2+1, ..., 3 (Section 2.2 coarsening by 2;
 * Table 2 caption: down to fewer than three unknowns per direction) and
 * allocate every coarse level and scratch buffer on the current device.
 * 'stream' is the hipStream_t all later work of this context goes to.
 * Errors: MG_EINVAL (null p/out, bad dim/n/nu/bc/op/smoother, var-coef without k),
 * MG_ENOMEM, MG_EDEVICE.  On error *out is NULL. */
int mg_setup(const mg_params* p, void* stream, mg_ctx** out);

/* Release every device buffer of the context (after finishing its work). NULL is a no-op. */
void mg_destroy(mg_ctx* ctx);

/* One V(nu1, nu2) cycle of Algorithm 1 on u (in/out, device) for rhs f (device).
 * With MG_PREC_FP32_IR it is one refinement step: r = f - A u (FP64), one FP32
 * V-cycle on A e = r from e = 0, u += e (FP64).  Asynchronous on the stream. */
int mg_vcycle(mg_ctx* ctx, double* u, const double* f);

/* Solve loop of the Layer-4 Application function: rho_0 = ||f - A u||_2, then
 * cycles (or refinement steps) until rho_k <= tol * rho_0 or max_cycles.
 * u: device, in (initial guess) / out.  cycles_done, res_hist: HOST pointers,
 * may be NULL; res_hist needs max_cycles + 1 doubles and receives rho_0..rho_k
 * (FP64 Euclidean norms over inner nodes).  Synchronises the stream.
 * Returns MG_OK, MG_ENOTCONV, MG_EDIVERGED (u then holds the last iterate). */
int mg_solve(mg_ctx* ctx, double* u, const double* f, double tol, int max_cycles, int* cycles_done,
             double* res_hist);

/* FP64 residual norm sqrt(sum over inner nodes of (f - A u)^2) into *out (HOST).
 * Synchronises the stream. */
int mg_residual_norm(mg_ctx* ctx, const double* u, const double* f, double* out);

/* Number of levels of the context's hierarchy (>= 1), or a negative status. */
int mg_num_levels(const mg_ctx* ctx);

/* Launch geometry the context uses on 'level' (0 = finest) for kernel 'family'
 * (0 smoothing, 1 residual + restriction, 2 finest-level norm / refinement
 * pass, 3 smoothing from a zero iterate, 4 smoothing with the coarse-grid
 * correction fused in, 5 the last pre-smoothing sweep fused with the residual
 * and restriction: *zchunk coarse planes per workgroup, 0 when the level runs
 * the sweep and the restriction apart, 6 (level 0 of an FP64 context) the
 * first pre-smoothing sweep that also sums the residual norm of its incoming
 * iterate, which in mg_solve gives each cycle's norm (Section 2.4's L2
 * residual; every field 0 when the norm is a pass of its own), 7 the first
 * two pre-smoothing sweeps from a zero iterate in one launch (mg_level_
 * smooth2_zero; *zchunk 0 when the level runs them apart), 8 the first two
 * post-smoothing sweeps in one launch (mg_level_smooth2_correct, 2D; *zchunk
 * 0 when the level runs them apart)): tile rows
 * *by, z-chunk *zchunk (3D planes per workgroup), for 3D
 * marching kernels *prefetch = planes of u loaded ahead (1 or 2), *waves =
 * wavefronts per workgroup (4; 1 or 8 for 3D smoothing and the 3D pass), for
 * smoothing *order = block-to-tile order (0: each XCD takes a contiguous band
 * of tiles, 1: linear), and for the pass *pairs = 1 if each lane holds two
 * adjacent nodes of a row (128-node-wide tiles, Laplacian only; in 2D *zchunk
 * is then the rows each wavefront marches); prefetch,
 * waves, order and pairs may be NULL.  These are the autotuner's choices
 * (measured at mg_setup unless the environment sets MG_AUTOTUNE=0) or the
 * built-in heuristic.  Results never depend on them. */
int mg_tile_config(const mg_ctx* ctx, int level, int family, int* by, int* zchunk, int* prefetch, int* waves,
                   int* order, int* pairs);

/* Human-readable name of a status code. */
const char* mg_strerror(int code);

/* ---------------------------------------------------------------------------
 * Single-level operations (one kernel each; the steps of Algorithm 1).  They
 * run one grid level with no context: dim 2/3, n = 2^L+1 >= 5 (n >= 3 for the
 * coarsest solve), dtype 0 = FP64 / 1 = FP32 for every array argument.
 * 'k' is null (Laplacian) or the nodal coefficient of this level.  'by' and
 * 'zchunk' pick the tile shape (0 = library default): by in {8, 16, 32},
 * zchunk >= 1 (3D only); 'prefetch' (3D smoothing) is 1 or 2 planes of u
 * loaded ahead and 'waves' (3D smoothing) 4 or 8 wavefronts per workgroup,
 * or 1: one wavefront per tile holding all of its rows in registers (by 8 or
 * 12) (0 = default).  3D sweeps hold by/waves rows per thread: at most 2 in
 * FP64 with a coefficient field, 4 in FP64 or with one, 8 otherwise; with one
 * wavefront, 12 rows
 * in FP32 without a coefficient field, 8 in FP32 with one or in FP64 without,
 * not available in FP64 with one (MG_EINVAL beyond).  'order' is the
 * block-to-tile order: 0 XCD bands, 1 linear.  Asynchronous on 'stream'.
 * ------------------------------------------------------------------------- */

/* One smoothing sweep (Section 2.4 GaussSeidel / Section 2.3 Jacobi) from u_in
 * to u_out (out of place; u_out's boundary is not written); smoother 2 is a
 * red-black sweep that relaxes black first (the post-smoothing sweep of
 * MG_SMOOTH_RBGS_SYM).  zero_guess != 0
 * treats u_in as identically zero (u_in may then be NULL).  ec, if not NULL,
 * is the coarse-grid correction ((n-1)/2+1 nodes per axis) added by
 * interpolation to u_in before the sweep (Algorithm 1: coarse-grid correction
 * followed by post-smoothing). */
int mg_level_smooth(int dim, int n, int dtype, int smoother, double omega, const void* k, const void* u_in,
                    const void* f, void* u_out, const void* ec, int zero_guess, int by, int zchunk, int prefetch,
                    int waves, int order, void* stream);

/* fc = full weighting of r = f - A u (Algorithm 1: residual and restriction)
 * on the inner nodes of the coarse grid ((n-1)/2+1 per axis); fc's boundary is not written. */
int mg_level_residual_restrict(int dim, int n, int dtype, const void* k, const void* u, const void* f, void* fc,
                               int by, int zchunk, void* stream);

/* u += P ec on inner fine nodes (Section 2.4 interpolatecorr; bilinear / trilinear P). */
int mg_level_prolong_correct(int dim, int n, int dtype, void* u, const void* ec, void* stream);

/* Coarsest grid (n = 3): u = f / diag at the single inner node. */
int mg_level_coarsest(int dim, int dtype, const void* k, void* u, const void* f, void* stream);

/* The last pre-smoothing sweep fused with the residual and full weighting
 * (Algorithm 1: presmoothing, residual, restriction), 3D Laplacian, dtype 1
 * (FP32) or 2 (binary16), omega 1: one red-first red-black sweep u_in -> u_out
 * (inner nodes; u_out != u_in) and fc (inner coarse nodes, edge (n-1)/2+1) =
 * full weighting of f - A u_out, bit for bit the sweep of mg_level_smooth
 * followed by mg_level_residual_restrict.  zchunk: coarse planes per
 * workgroup (>= 1); order: 0 XCD bands, 1 linear block order.  The solver
 * uses it in V-cycles where the autotuner times it faster than the two
 * kernels it replaces.  Synchronises the stream. */
int mg_level_smooth_restrict(int dim, int n, int dtype, const void* u_in, const void* f, void* u_out, void* fc,
                             int zchunk, int order, void* stream);
/* The first two pre-smoothing sweeps of a level whose iterate starts at zero
 * (Algorithm 1: presmoothing from the zero coarse-grid guess), fused,
 * Laplacian, dtype 1 (FP32) or 2 (binary16), omega 1: two red-first
 * red-black sweeps from u = 0, the result in u_out (inner nodes; f != u_out),
 * bit for bit mg_level_smooth with zero_guess followed by mg_level_smooth.
 * 3D: by 12 or 16 rows per tile (the tile writes (64 - 6) x (by - 6) nodes
 * per plane), zchunk planes per workgroup; 2D: by ignored, zchunk rows per
 * wavefront (strips of 128 nodes, two per lane, writing 122 per row); zchunk >= 1; order: 0
 * XCD bands, 1 linear block order.  The solver uses it in V-cycles (and
 * batches) where the autotuner times it faster than the two sweeps it
 * replaces.  Synchronises the stream. */
int mg_level_smooth2_zero(int dim, int n, int dtype, const void* f, void* u_out, int by, int zchunk, int order,
                          void* stream);
/* The first two post-smoothing sweeps of a level (Algorithm 1: interpolation
 * and correction, then postsmoothing), fused, 2D Laplacian, dtype 1 (FP32) or
 * 2 (binary16), omega 1: the bilinear correction from the coarse grid ec
 * (edge (n-1)/2+1) added to u_in at inner nodes, then two red-black sweeps
 * (smoother 0: red first; 2: black first, the symmetric smoother's order),
 * the result in u_out (inner nodes; u_out != u_in), bit for bit
 * mg_level_smooth with ec followed by mg_level_smooth.  zchunk: rows per
 * wavefront (strips of 128 nodes, two per lane, writing 120 per row); order: 0 XCD bands, 1
 * linear block order.  The solver uses it in V-cycles (and batches) where the
 * autotuner times it faster than the two sweeps it replaces.  Synchronises
 * the stream. */
int mg_level_smooth2_correct(int dim, int n, int dtype, int smoother, const void* u_in, const void* f,
                             const void* ec, void* u_out, int zchunk, int order, void* stream);
/* Conjugate gradients on a coarsest grid of n = 2^c + 1 nodes per axis
 * (mg_params.coarse_n): 'iters' steps (0: 4 (n - 1)) from u = 0 on A u = f;
 * u's boundary is written with zeros.  n at most 33 (2D) / 9 (3D) for dtype 0,
 * 65 / 17 otherwise (MG_ENOTSUP beyond). */
int mg_level_coarsest_cg(int dim, int n, int dtype, const void* k, void* u, const void* f, int iters,
                         void* stream);

/* ---------------------------------------------------------------------------
 * Complex diffusion (Section 4, Eq. (2)): u_t = div(g(Im u) grad u) on the unit
 * square / cube with a homogeneous Neumann boundary, complex diffusivity
 * g(s) = e^{i theta} / (1 + (s / (k theta))^2); averaged finite differences on
 * a cell-centred grid of n = 2^L cells per axis (face diffusivity = mean of the
 * two cells' g; a face on the boundary carries no flux), implicit Euler in
 * time, and per time step the full approximation scheme (FAS) with lagged
 * diffusivity (each smoothing sweep and each residual uses g of the iterate
 * it starts from), averaging restriction of the residual and of the full
 * approximation, constant interpolation of the coarse correction, a single-
 * cell coarsest level solved exactly.  Complex arrays are device arrays of
 * n^dim (re, im) FP64 pairs, x fastest, 16-byte aligned (MG_EINVAL otherwise).
 * ------------------------------------------------------------------------- */
typedef struct mg_cdiff_params {
    int dim;        /* 2 or 3 */
    int n;          /* cells per axis, 2^L, L >= 1 (at most 4096 in 2D, 256 in 3D) */
    double tau;     /* time step, > 0 */
    double theta;   /* angle of the diffusivity, 0 < theta < pi/2 */
    double k;       /* scaling parameter, > 0 */
    int smoother;   /* MG_SMOOTH_RBGS or MG_SMOOTH_WJACOBI */
    double omega;   /* <= 0: 1.0 (RBGS) / 0.8 (Jacobi) */
    int nu1, nu2;   /* smoothing sweeps, 0..16 */
} mg_cdiff_params;

/* Build the hierarchy (n, n/2, ..., 1 cells per axis) and its work arrays on
 * the current device; cos theta and sin theta are evaluated once here.
 * Errors: MG_EINVAL, MG_ENOMEM, MG_EDEVICE.  Release with mg_destroy. */
int mg_cdiff_setup(const mg_cdiff_params* p, void* stream, mg_ctx** out);
/* One FAS cycle on u (in/out) for N(u) = f, N(u) = u / tau - div(g(Im u) grad u).
 * Asynchronous. */
int mg_cdiff_fas(mg_ctx* ctx, double* u, const double* f);
/* out = N(u). Asynchronous. */
int mg_cdiff_apply(mg_ctx* ctx, const double* u, double* out);
/* 'steps' implicit-Euler steps on u (in: u^0, out: u^steps); step m solves
 * N(u) = u^m / tau by FAS cycles from u^m until ||f - N(u)|| <= tol ||f - N(u^m)||
 * or max_cycles.  cycles (HOST, may be NULL) receives each step's cycle count,
 * res_hist (HOST, may be NULL, steps * (max_cycles + 1) doubles) each step's
 * residual norms (row m starts at m * (max_cycles + 1)).  Synchronises the
 * stream.  Returns MG_OK, or MG_ENOTCONV if a step missed the tolerance. */
int mg_cdiff_run(mg_ctx* ctx, double* u, int steps, double tol, int max_cycles, int* cycles, double* res_hist);

/* Constant stencil (MG_OP_CONST_STENCIL), FP64, node grids of n = 2^L + 1
 * nodes per axis; 'stencil' is a HOST pointer to 2*dim + 1 coefficients
 * (centre first, > 0, then -x, +x, -y, +y[, -z, +z]).  One smoothing sweep
 * u_in -> u_out (smoother 0 RBGS red first, 1 Jacobi (u_out != u_in), 2
 * RBGS black first; omega <= 0: 1.0 / 0.8); fc (inner coarse nodes, edge
 * (n-1)/2+1, n >= 5) = full weighting of f - A u; and the exact solve of the
 * single unknown of a 3-node grid, u = f / (c s0).  Asynchronous. */
int mg_level_st_smooth(int dim, int n, const double* stencil, int smoother, double omega, const double* u_in,
                       const double* f, double* u_out, void* stream);
int mg_level_st_residual_restrict(int dim, int n, const double* stencil, const double* u, const double* f,
                                  double* fc, void* stream);
int mg_level_st_coarsest(int dim, const double* stencil, double* u, const double* f, void* stream);

/* Cell-centred Neumann grids (MG_BC_NEUMANN_CC), FP64, n = 2^L cells per axis
 * (n >= 2), the operations of a cycle: one smoothing sweep u_in -> u_out
 * (smoother 0 RBGS red first, 1 Jacobi); fc = average of the children's
 * residuals (n/2 cells per axis); u += constant interpolation of ec; and
 * v -= mean(v), *mean_out (HOST) = the mean removed (sum in the fixed order:
 * each x-row, the rows of a plane, the planes).  The first three are
 * asynchronous; the last synchronises the stream. */
int mg_level_cc_smooth(int dim, int n, int smoother, double omega, const double* u_in, const double* f,
                       double* u_out, void* stream);
int mg_level_cc_residual_restrict(int dim, int n, const double* u, const double* f, double* fc, void* stream);
int mg_level_cc_prolong_correct(int dim, int n, double* u, const double* ec, void* stream);
int mg_level_cc_remove_mean(int dim, int n, double* v, double* mean_out, void* stream);

/* dtype 2 in the four calls above: binary16 arrays (u, f, the coarse arrays),
 * arithmetic in FP32, each value the method stores rounded to binary16 (the
 * fields of MG_PREC_FP16_IR); Laplacian only (k must be NULL, else
 * MG_ENOTSUP). */

/* FP64 refinement pass: u_out = u_in + e on inner nodes, r = (float)(f - A u_out)
 * on inner nodes (FP64 operator, FP64 k or NULL), *norm_out (HOST) = ||f - A u_out||_2.
 * e and r are FP32 arrays; u_out's and r's boundaries are not written.  'by',
 * 'zchunk' pick the tile (0 = default); in 3D 'prefetch' is 1 or 2 planes
 * loaded ahead and 'waves' 4 or 8 wavefronts per workgroup (8 needs
 * by >= 16); 0 = default; 'pairs' != 0 (k NULL) runs the variant with two
 * adjacent nodes per lane (128 nodes per tile row; 3D: by <= 4 * waves, else
 * MG_EINVAL; 2D: each of four wavefronts marches 'zchunk' rows along y, 0 =
 * 32, by ignored).  Synchronises the stream. */
int mg_level_ir_update(int dim, int n, const double* k, const double* u_in, const float* e, const double* f,
                       double* u_out, float* r, double* norm_out, int by, int zchunk, int prefetch, int waves,
                       int pairs, void* stream);

/* Refinement pass of MG_PREC_FP16_IR (Laplacian): when e16 (binary16, the
 * correction scaled by e_scale, a power of two) is not NULL, u_out = u_in +
 * e16 / e_scale on inner nodes, else u_out is not written and the pass reads
 * u_in; r = f - A u in FP64; r16 (binary16) = half(float(s) * float(r)) on
 * inner nodes, s the power of two with 8 <= s * prev_max < 16 and exponent
 * within -126 .. 127 (1 if prev_max is 0 or not finite); *norm_out = ||r||_2
 * and *max_out = max |r| (HOST).
 * Two nodes per lane: 3D tiles by x waves of 8x4 / 16x4 / 16x8 / 32x8, 2D
 * 'zchunk' rows per wavefront (0 = 32).  Synchronises the stream. */
int mg_level_ir_update_f16(int dim, int n, const double* u_in, const void* e16, double e_scale, double prev_max,
                           const double* f, double* u_out, void* r16, double* norm_out, double* max_out, int by,
                           int zchunk, int prefetch, int waves, void* stream);

/* The refinement pass of mg_level_ir_update (same arguments, same kernels,
 * same results bit for bit) for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  It calls no hipMalloc / hipFree and no allocating library
 * routine: its scratch (launch descriptor, one FP64 norm partial per
 * workgroup, the finalized norm) is a static 1 MiB device array that each
 * device holds from the library's first use on it until the process ends.
 * Launch shapes with more than 131008 workgroups (norm partials) are rejected
 * with MG_ENOMEM before anything is enqueued (the default shapes stay far
 * below: 3D n = 1025 needs about 1.1e4).  Every call on one device uses the
 * same array: calls that overlap on one device (other streams or host
 * threads) race and must be serialised by the caller.  Synchronises the
 * stream. */
int mg_level_ir_update_noalloc(int dim, int n, const double* k, const double* u_in, const float* e,
                               const double* f, double* u_out, float* r, double* norm_out, int by, int zchunk,
                               int prefetch, int waves, int pairs, void* stream);

/* ---------------------------------------------------------------------------
 * Batched solves: many independent grids (sizes may differ) in one context.
 * Every instance is solved with FP32 V-cycles inside FP64 refinement; each V-cycle
 * step is one launch per grid level shared by every instance that has that level,
 * so instances of different sizes join the descending leg at their own finest
 * level.  Each instance stops on its own residual test (a device-side flag);
 * its result is bitwise identical to solving it alone with mg_solve.
 * ------------------------------------------------------------------------- */

/* count instances, each[i] their parameters: same dim, smoother, omega, nu1, nu2 for
 * all; precision MG_PREC_FP32_IR; op MG_OP_LAPLACE (MG_ENOTSUP otherwise); n may differ.
 * Allocates every instance's hierarchy and, unless the environment sets
 * MG_AUTOTUNE=0, times the tile geometries of each level's batched launches
 * on them (results never depend on the choice).  Destroy with mg_destroy. */
int mg_batch_setup(int count, const mg_params* each, void* stream, mg_ctx** out);

/* u[i], f[i]: DEVICE pointers (host array of count pointers) of instance i, as in
 * mg_solve.  cycles_done[i] / status[i] (HOST, may be NULL) receive each instance's
 * refinement steps and status (MG_OK, MG_ENOTCONV, MG_EDIVERGED).  Returns the worst
 * status.  Synchronises the stream. */
int mg_batch_solve(mg_ctx* ctx, double* const* u, const double* const* f, double tol, int max_cycles,
                   int* cycles_done, int* status);

/* ---------------------------------------------------------------------------
 * Serving: a request loop with continuous batching.  Requests (2D or 3D grids
 * of any accepted size) are queued; each mg_server_step admits queued requests
 * in arrival order while a slot and the HBM budget allow (hierarchies are kept
 * resident and reused from a per-size pool; the right-hand side is uploaded on
 * a copy stream of the server and the request joins once it has landed),
 * queues one refinement step (FP32 V-cycle + FP64 pass) of every joined
 * request in shared per-level launches, and completes the requests whose
 * residual test passed in the previous step (steps are pipelined: the call
 * returns while the step it queued runs; results are copied back on the copy
 * stream).
 * ------------------------------------------------------------------------- */

typedef struct mg_server_params {
    size_t hbm_budget_bytes; /* device bytes request hierarchies may hold (pool included) */
    int max_slots;           /* concurrent requests per dimension */
    int max_n2d, max_n3d;    /* largest accepted edges (2^L+1; at most 32769 / 1025) */
    int smoother;            /* enum mg_smoother */
    double omega;            /* <= 0: paper's value */
    int nu1, nu2;            /* 0, 0 selects V(2,2) */
    double tol;              /* relative residual reduction of every request */
    int max_cycles;          /* refinement steps before a request completes unconverged */
} mg_server_params;

int mg_server_create(const mg_server_params* sp, void* stream, mg_ctx** out);
/* Queue a request: dim 2/3, n = 2^L+1 (5 <= n <= max edge), f_host: HOST array of n^dim
 * doubles (copied).  MG_ENOMEM if the request alone exceeds the budget. */
int mg_server_submit(mg_ctx* ctx, int dim, int n, const double* f_host, long long* req_id);
/* Queue a request whose data stay in device memory: f_dev (DEVICE, n^dim
 * doubles, caller-owned, complete before the call) is copied device to device
 * when the request is admitted and must stay unchanged until the request is
 * reported done; the solution is copied into u_dev (DEVICE, n^dim doubles,
 * caller-owned) on the server's copy stream and is there once mg_server_poll
 * has reported the request.  mg_server_fetch then returns its statistics
 * (u_host must be NULL for such a request).  Errors as mg_server_submit. */
int mg_server_submit_device(mg_ctx* ctx, int dim, int n, const double* f_dev, double* u_dev, long long* req_id);
/* Admit, queue one refinement step of every joined request, complete the ones
 * the previous step finished.  Waits for the previous step only (not for the
 * one it queues); the queued step runs on the server's stream.  n_active
 * (admitted, not yet completed) / n_queued (HOST, may be NULL) after the call. */
int mg_server_step(mg_ctx* ctx, int* n_active, int* n_queued);
/* Ids of requests completed (result copied to host memory) since the last poll
 * (up to cap) into done_ids (HOST).  Does not wait. */
int mg_server_poll(mg_ctx* ctx, long long* done_ids, int cap, int* ndone);
/* Result of a completed request: u_host (n^dim doubles, may be NULL), refinement steps,
 * final ||r||/||r0|| and seconds from submit to completion.  The request is released.
 * Returns its status, or MG_EBUSY if it has not completed. */
int mg_server_fetch(mg_ctx* ctx, long long req_id, double* u_host, int* cycles, double* final_rel_res,
                    double* latency_s);
/* Device bytes held (active + pooled hierarchies), active and queued requests. */
int mg_server_info(mg_ctx* ctx, size_t* used_bytes, int* active, int* queued);

/* ---------------------------------------------------------------------------
 * Measurement hooks.
 * ------------------------------------------------------------------------- */

/* When on, mg_solve runs without graph capture and brackets two kernels of
 * every refinement step (or cycle) with HIP events on the context's stream:
 * kernel 0, the finest-level smoothing sweeps that read the previous iterate
 * (not the zero-iterate or fused-correction variants); kernel 1, the
 * finest-level FP64 refinement pass (mixed precision) or norm pass (FP64).
 * Launches of steps past the solve's last step (queued before the stop test
 * was read; they find the stop flag set and do no work) are not counted.
 * mg_prof_read_kernel returns the number of counted launches of one kernel
 * and their summed duration in ms since the last read, and resets them;
 * mg_prof_read is kernel 0.  MG_EINVAL for a batch or server handle or
 * another kernel number. */
int mg_prof_enable(mg_ctx* ctx, int on);
int mg_prof_read_kernel(mg_ctx* ctx, int kernel, int* launches, double* total_ms);
int mg_prof_read(mg_ctx* ctx, int* launches, double* total_ms);

/* Plain device-to-device copy kernel of 'bytes' bytes (multiple of 16):
 * calibration of the HBM traffic counters against a known byte count. */
int mg_copy_kernel(void* dst, const void* src, size_t bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* MG_H */
