/*
 * oracle.cpp -- plain CPU reference of the geometric multigrid V-cycle.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  The product library shares
 * no source with it and never calls it.
 *
 * What it computes (Koestler et al., arXiv:1406.5369):
 *   - Section 2.1, Eq. (1): Poisson's equation with homogeneous Dirichlet
 *     boundary on the unit square / cube, solved here in the form -Lap u = f
 *     (the symmetric positive definite sign; the smoother formula of
 *     Section 2.4 is sign-agnostic because it divides by the diagonal of the
 *     same operator).
 *   - Section 2.2: node-based grids, second-order finite differences, a
 *     constant 5-point (2D) / 7-point (3D) stencil, coarsening by 2 per axis.
 *     A grid has n = 2^L + 1 nodes per axis including the boundary and
 *     spacing h = 1/(n-1); levels are coarsened down to n = 3 (one unknown
 *     per axis), as in the caption of Table 2.
 *   - Section 2.3, Algorithm 1: the recursive V-cycle (correction scheme):
 *     presmooth, residual, restriction, recursion from a zero guess,
 *     prolongation and correction, postsmooth; exact solve on the coarsest
 *     grid (one unknown: u = f / diag).
 *   - Section 2.3 component list and Table 1: omega-Jacobi and red-black
 *     Gauss-Seidel smoothers, "direct" coarse operators (the stencil is
 *     re-discretised with the coarse spacing), full-weighting restriction
 *     and bi-/trilinear interpolation.
 *   - Section 2.4 (Layer-4 functions GaussSeidel, Restrict, interpolatecorr,
 *     VCycle, Application): the update u + omega * diag^-1 (f - A u) on inner
 *     points, red points first, the solve loop that prints the L2 residual
 *     after every cycle.
 *   - Section 4 / Table 2 caption: omega = 0.8 for Jacobi, 1.0 for RBGS.
 *   - Table 1 "single/double accuracy": the same algorithm instantiated in
 *     float (used as the inner solver of FP64 iterative refinement).
 *
 * Readings taken where the paper is silent (each also fixed on the HIP side):
 *   - colour of node (i,j[,k]) is (i+j[+k]) mod 2; red = 0 is updated first
 *     in every sweep, pre- and post-smoothing alike;
 *   - full weighting is the tensor product of (1/4, 1/2, 1/4) per axis, and
 *     the interpolation is bilinear / trilinear (weights 1, 1/2, 1/4, 1/8),
 *     i.e. P = 2^d R^T;
 *   - every operation touches inner nodes only; boundary nodes stay 0;
 *   - the residual norm is the unscaled Euclidean norm over inner nodes;
 *   - per-point expressions are written in one fixed evaluation order (below)
 *     and compiled without floating-point contraction, so that any other
 *     implementation writing the same expressions rounds identically.
 *
 * Variable coefficients (-div(k grad u) = f, 7-/5-point flux form): the face
 * coefficient between nodes p and q is the harmonic mean 2 k_p k_q/(k_p+k_q);
 * coarse k is taken by injection k_{l+1}(I) = k_l(2I) and the operator is
 * re-discretised on every level (Table 1, "direct (re-discretization)").
 *
 * Constant stencil (Section 2.2: the discretisation is a stencil declared
 * with constant entries; the Laplacian's 5-/7-point stencil is one choice):
 * (A u)_p = (1/h^2) (s0 u_p + sW u_W + sE u_E + sS u_S + sN u_N [+ sB u_B + sT u_T]),
 * coefficients given centre first, then -x, +x, -y, +y[, -z, +z]; the same
 * stencil on every level with that level's h ("direct" coarse operators).
 *
 * Layout: x fastest, idx = (k*n + j)*n + i (3D) or j*n + i (2D).
 */
#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

typedef std::ptrdiff_t idx_t;

/* ------------------------------------------------------------------ */
/* Storage types.  FP64 and FP32 hierarchies compute in their storage    */
/* type; the half-precision hierarchy stores IEEE 754 binary16 values and */
/* computes in float (Table 1's data-type choice taken one step below    */
/* single precision, for storage only).                                  */
/* ------------------------------------------------------------------ */

/* binary16 bits -> float (exact): 1 sign bit, 5 exponent bits (bias 15),
 * 10 fraction bits; exponent 0 holds the subnormals fraction * 2^-24. */
inline float half_to_float(uint16_t h) {
    const int sign = (h >> 15) & 1, ex = (h >> 10) & 31, fr = h & 1023;
    double a;
    if (ex == 0) a = std::ldexp((double)fr, -24);
    else if (ex == 31) a = fr ? NAN : INFINITY;
    else a = std::ldexp((double)(1024 + fr), ex - 25);
    return (float)(sign ? -a : a);
}

/* float -> nearest binary16 (ties to even), by the definition: below 2^-14
 * the representable values are the multiples of 2^-24; in the binade
 * [2^E, 2^(E+1)) they are the multiples of 2^(E-10); magnitudes from 65520
 * on (half-way between the largest finite value 65504 and 2^16) become
 * infinity.  std::nearbyint rounds to the nearest integer, ties to even, in
 * the default rounding mode. */
inline uint16_t float_to_half(float x) {
    if (std::isnan(x)) return 0x7e00;
    const uint16_t sign = std::signbit(x) ? 0x8000 : 0;
    const double a = std::fabs((double)x);
    if (a >= 65520.0) return (uint16_t)(sign | 0x7c00);
    if (a < std::ldexp(1.0, -14)) return (uint16_t)(sign | (uint16_t)std::nearbyint(std::ldexp(a, 24)));
    int e;
    (void)std::frexp(a, &e); /* a = m 2^e, 1/2 <= m < 1: leading bit 2^(e-1) */
    int E = e - 1;
    double q = std::nearbyint(std::ldexp(a, 10 - E)); /* 1024 .. 2048 */
    if (q == 2048.0) {
        q = 1024.0;
        ++E;
    }
    return (uint16_t)(sign | (uint16_t)((E + 15) << 10) | (uint16_t)(q - 1024.0));
}

/* A binary16 storage cell: stores the rounded value of what is assigned to
 * it, reads back as float. */
struct Half {
    uint16_t bits;
    Half() = default;
    Half(float x) : bits(float_to_half(x)) {}
    operator float() const { return half_to_float(bits); }
};
static_assert(sizeof(Half) == 2, "binary16 cells are two bytes");

template <typename S>
struct Arith {
    typedef S type;
};
template <>
struct Arith<Half> {
    typedef float type;
};

/* ------------------------------------------------------------------ */
/* Per-point operator: (A u)_p for inner node p.                        */
/* ------------------------------------------------------------------ */

template <typename S>
struct Grid {
    typedef typename Arith<S>::type T;
    int dim;      /* 2 or 3 */
    int n;        /* nodes per axis, boundary included */
    T c;          /* 1/h^2 in working precision */
    T wd;         /* omega*h^2/(2d): inverse diagonal times omega (Poisson) */
    T omega;      /* smoother weight */
    const T* k;   /* nodal coefficient (variable coefficients), in the arithmetic type, or nullptr */
    const T* st = nullptr; /* constant stencil (2d+1 entries, centre first), or nullptr */
};

/* harmonic-mean face coefficient between nodes with values a and b */
template <typename T>
inline T kface(T a, T b) {
    return ((T(2) * a) * b) / (a + b);
}

/* Poisson: (A u)_p = c * (2d u_p - sum of neighbours), fixed summation order */
template <typename S>
inline typename Arith<S>::type apply_poisson(const Grid<S>& g, const S* u, idx_t p) {
    typedef typename Arith<S>::type T;
    const idx_t sx = 1, sy = g.n, sz = (idx_t)g.n * g.n;
    const T uC = u[p];
    if (g.dim == 2) {
        const T s = (u[p - sx] + u[p + sx]) + (u[p - sy] + u[p + sy]);
        return g.c * (T(4) * uC - s);
    }
    const T s = ((u[p - sx] + u[p + sx]) + (u[p - sy] + u[p + sy])) + (u[p - sz] + u[p + sz]);
    return g.c * (T(6) * uC - s);
}

/* Variable coefficients: (A u)_p = c * (dsum u_p - t); also returns dsum */
template <typename S>
inline typename Arith<S>::type apply_varcoef(const Grid<S>& g, const S* u, idx_t p, typename Arith<S>::type* dsum_out) {
    typedef typename Arith<S>::type T;
    const idx_t sx = 1, sy = g.n, sz = (idx_t)g.n * g.n;
    const T* k = g.k;
    const T kp = k[p];
    const T kxW = kface(k[p - sx], kp), kxC = kface(kp, k[p + sx]);
    const T kyS = kface(k[p - sy], kp), kyC = kface(kp, k[p + sy]);
    T dsum, t;
    if (g.dim == 2) {
        dsum = (kxW + kxC) + (kyS + kyC);
        t = (kxW * u[p - sx] + kxC * u[p + sx]) + (kyS * u[p - sy] + kyC * u[p + sy]);
    } else {
        const T kzB = kface(k[p - sz], kp), kzC = kface(kp, k[p + sz]);
        dsum = ((kxW + kxC) + (kyS + kyC)) + (kzB + kzC);
        t = ((kxW * u[p - sx] + kxC * u[p + sx]) + (kyS * u[p - sy] + kyC * u[p + sy])) +
            (kzB * u[p - sz] + kzC * u[p + sz]);
    }
    *dsum_out = dsum;
    return g.c * (dsum * u[p] - t);
}

/* Constant stencil: (A u)_p = c * (s0 u_p + t), t the weighted neighbours
 * paired as ((W+E)+(S+N))+(B+T) */
template <typename S>
inline typename Arith<S>::type apply_stencil(const Grid<S>& g, const S* u, idx_t p) {
    typedef typename Arith<S>::type T;
    const idx_t sx = 1, sy = g.n, sz = (idx_t)g.n * g.n;
    const T* a = g.st;
    T t = (a[1] * u[p - sx] + a[2] * u[p + sx]) + (a[3] * u[p - sy] + a[4] * u[p + sy]);
    if (g.dim == 3) t = t + (a[5] * u[p - sz] + a[6] * u[p + sz]);
    return g.c * (a[0] * u[p] + t);
}

/* residual r_p = f_p - (A u)_p */
template <typename S>
inline typename Arith<S>::type residual_at(const Grid<S>& g, const S* u, const S* f, idx_t p) {
    typedef typename Arith<S>::type T;
    if (g.st) return f[p] - apply_stencil(g, u, p);
    if (g.k) {
        T dsum;
        const T Au = apply_varcoef(g, u, p, &dsum);
        return f[p] - Au;
    }
    return f[p] - apply_poisson(g, u, p);
}

/* smoother update of Section 2.4: u + omega * diag^-1 * (f - A u) */
template <typename S>
inline typename Arith<S>::type smooth_at(const Grid<S>& g, const S* u, const S* f, idx_t p) {
    typedef typename Arith<S>::type T;
    if (g.k) {
        T dsum;
        const T Au = apply_varcoef(g, u, p, &dsum);
        const T r = f[p] - Au;
        return u[p] + (g.omega * r) / (g.c * dsum);
    }
    /* constant stencils: wd = omega h^2 / s0 (the Laplacian's s0 = 2d) */
    const T r = f[p] - (g.st ? apply_stencil(g, u, p) : apply_poisson(g, u, p));
    return u[p] + g.wd * r;
}

/* loops over inner nodes: (outer index, inner linear index) */
inline idx_t at(int dim, int n, int i, int j, int k) {
    return dim == 2 ? (idx_t)j * n + i : ((idx_t)k * n + j) * n + i;
}

/* ------------------------------------------------------------------ */
/* Smoothers (Section 2.3 component list; Section 2.4 GaussSeidel)      */
/* ------------------------------------------------------------------ */

/* One red-black Gauss-Seidel sweep in place: all red nodes, then all black
 * (first = 1: all black, then all red -- the second half of a symmetric
 * red-black smoother, Table 1 "red-black variants"). */
template <typename S>
void rbgs_sweep(const Grid<S>& g, S* u, const S* f, int first = 0) {
    const int n = g.n;
    const int k0 = g.dim == 3 ? 1 : 0, k1 = g.dim == 3 ? n - 1 : 1; /* one pass of k in 2D */
    for (int half = 0; half < 2; ++half) {
        const int colour = half ^ first;
#pragma omp parallel for schedule(static)
        for (int k = k0; k < k1; ++k)
            for (int j = 1; j < n - 1; ++j)
                for (int i = 1; i < n - 1; ++i) {
                    if (((i + j + k) & 1) != colour) continue; /* k = 0 in 2D */
                    const idx_t p = at(g.dim, n, i, j, k);
                    u[p] = smooth_at(g, u, f, p);
                }
    }
}

/* One omega-Jacobi sweep: every new value from old values only. */
template <typename S>
void jacobi_sweep(const Grid<S>& g, S* u, const S* f, std::vector<S>& tmp) {
    const int n = g.n;
    const size_t total = g.dim == 3 ? (size_t)n * n * n : (size_t)n * n;
    tmp.assign(u, u + total);
    const int k0 = g.dim == 3 ? 1 : 0, k1 = g.dim == 3 ? n - 1 : 1;
#pragma omp parallel for schedule(static)
    for (int k = k0; k < k1; ++k)
        for (int j = 1; j < n - 1; ++j)
            for (int i = 1; i < n - 1; ++i) {
                const idx_t p = at(g.dim, n, i, j, k);
                tmp[p] = smooth_at(g, u, f, p);
            }
    std::memcpy(u, tmp.data(), total * sizeof(S));
}

/* r = f - A u on inner nodes, 0 on the boundary (Algorithm 1, residual) */
template <typename S>
void residual(const Grid<S>& g, const S* u, const S* f, typename Arith<S>::type* r) {
    typedef typename Arith<S>::type T;
    const int n = g.n;
    const size_t total = g.dim == 3 ? (size_t)n * n * n : (size_t)n * n;
    std::memset(r, 0, total * sizeof(T));
    const int k0 = g.dim == 3 ? 1 : 0, k1 = g.dim == 3 ? n - 1 : 1;
#pragma omp parallel for schedule(static)
    for (int k = k0; k < k1; ++k)
        for (int j = 1; j < n - 1; ++j)
            for (int i = 1; i < n - 1; ++i) {
                const idx_t p = at(g.dim, n, i, j, k);
                r[p] = residual_at(g, u, f, p);
            }
}

/* Unscaled Euclidean norm of f - A u over inner nodes, summed in FP64.
 * Partial sums per outer index, then added in index order (deterministic
 * whatever the thread count). */
template <typename S>
double residual_norm(const Grid<S>& g, const S* u, const S* f) {
    const int n = g.n;
    const int k0 = g.dim == 3 ? 1 : 0, k1 = g.dim == 3 ? n - 1 : 1;
    std::vector<double> part((size_t)n, 0.0);
#pragma omp parallel for schedule(static)
    for (int k = k0; k < k1; ++k) {
        double s = 0.0;
        for (int j = 1; j < n - 1; ++j)
            for (int i = 1; i < n - 1; ++i) {
                const double r = (double)residual_at(g, u, f, at(g.dim, n, i, j, k));
                s += r * r;
            }
        part[(size_t)k] = s;
    }
    double s = 0.0;
    for (int k = k0; k < k1; ++k) s += part[(size_t)k];
    return std::sqrt(s);
}

/* ------------------------------------------------------------------ */
/* Inter-grid transfers (Section 2.3: full weighting and its partner    */
/* bilinear/trilinear interpolation; Section 2.4 Restrict, interpolatecorr) */
/* ------------------------------------------------------------------ */

/* fc(I) = sum over the 3^d fine neighbours of 2I of w(delta) r(2I+delta),
 * w = prod_a 2^-|delta_a| / 2^d; coarse boundary set to 0. */
template <typename S>
void restrict_fw(int dim, int nf, const typename Arith<S>::type* r, S* fc) {
    typedef typename Arith<S>::type T;
    const int nc = (nf - 1) / 2 + 1;
    const size_t total = dim == 3 ? (size_t)nc * nc * nc : (size_t)nc * nc;
    std::memset(fc, 0, total * sizeof(S));
    const idx_t sx = 1, sy = nf, sz = (idx_t)nf * nf;
    const int K0 = dim == 3 ? 1 : 0, K1 = dim == 3 ? nc - 1 : 1;
#pragma omp parallel for schedule(static)
    for (int K = K0; K < K1; ++K)
        for (int J = 1; J < nc - 1; ++J)
            for (int I = 1; I < nc - 1; ++I) {
                const idx_t q = at(dim, nc, I, J, K);
                if (dim == 2) {
                    const idx_t p = at(2, nf, 2 * I, 2 * J, 0);
                    const T edges = (r[p - sx] + r[p + sx]) + (r[p - sy] + r[p + sy]);
                    const T corners = (r[p - sx - sy] + r[p + sx - sy]) + (r[p - sx + sy] + r[p + sx + sy]);
                    fc[q] = (T(0.25) * r[p] + T(0.125) * edges) + T(0.0625) * corners;
                } else {
                    const idx_t p = at(3, nf, 2 * I, 2 * J, 2 * K);
                    const T faces = ((r[p - sx] + r[p + sx]) + (r[p - sy] + r[p + sy])) + (r[p - sz] + r[p + sz]);
                    const T exy = (r[p - sx - sy] + r[p + sx - sy]) + (r[p - sx + sy] + r[p + sx + sy]);
                    const T exz = (r[p - sx - sz] + r[p + sx - sz]) + (r[p - sx + sz] + r[p + sx + sz]);
                    const T eyz = (r[p - sy - sz] + r[p + sy - sz]) + (r[p - sy + sz] + r[p + sy + sz]);
                    const T edges = (exy + exz) + eyz;
                    const T cz0 = (r[p - sx - sy - sz] + r[p + sx - sy - sz]) + (r[p - sx + sy - sz] + r[p + sx + sy - sz]);
                    const T cz1 = (r[p - sx - sy + sz] + r[p + sx - sy + sz]) + (r[p - sx + sy + sz] + r[p + sx + sy + sz]);
                    const T corners = cz0 + cz1;
                    fc[q] = ((T(0.125) * r[p] + T(0.0625) * faces) + T(0.03125) * edges) + T(0.015625) * corners;
                }
            }
}

/* Interpolated coarse value at fine node (i,j,k): bilinear / trilinear.
 * Along an odd axis the node lies midway between coarse nodes I and I+1. */
template <typename S>
typename Arith<S>::type interp_at(int dim, int nc, const S* e, int i, int j, int k) {
    typedef typename Arith<S>::type T;
    const int I = i / 2, J = j / 2, K = k / 2;
    const int oi = i & 1, oj = j & 1, ok = dim == 3 ? (k & 1) : 0;
    const idx_t sx = 1, sy = nc, sz = (idx_t)nc * nc;
    const idx_t q = at(dim, nc, I, J, K);
    /* collect the strides of the odd axes in x, y, z order */
    idx_t s[3];
    int m = 0;
    if (oi) s[m++] = sx;
    if (oj) s[m++] = sy;
    if (ok) s[m++] = sz;
    if (m == 0) return e[q];
    if (m == 1) return T(0.5) * (e[q] + e[q + s[0]]);
    if (m == 2) return T(0.25) * ((e[q] + e[q + s[0]]) + (e[q + s[1]] + e[q + s[0] + s[1]]));
    return T(0.125) * (((e[q] + e[q + s[0]]) + (e[q + s[1]] + e[q + s[0] + s[1]])) +
                       ((e[q + s[2]] + e[q + s[0] + s[2]]) + (e[q + s[1] + s[2]] + e[q + s[0] + s[1] + s[2]])));
}

/* u_fine += P e_coarse on inner fine nodes */
template <typename S>
void prolong_correct(int dim, int nf, S* u, const S* ec) {
    const int nc = (nf - 1) / 2 + 1;
    const int k0 = dim == 3 ? 1 : 0, k1 = dim == 3 ? nf - 1 : 1;
#pragma omp parallel for schedule(static)
    for (int k = k0; k < k1; ++k)
        for (int j = 1; j < nf - 1; ++j)
            for (int i = 1; i < nf - 1; ++i) {
                const idx_t p = at(dim, nf, i, j, k);
                u[p] = u[p] + interp_at(dim, nc, ec, i, j, k);
            }
}

/* Coarsest grid n = 3: a single unknown, solved exactly: u = f / diag. */
template <typename S>
void coarsest_solve(const Grid<S>& g, S* u, const S* f) {
    typedef typename Arith<S>::type T;
    const idx_t p = at(g.dim, 3, 1, 1, 1);
    T diag;
    if (g.st) {
        diag = g.c * g.st[0];
    } else if (g.k) {
        T dsum;
        (void)apply_varcoef(g, u, p, &dsum);
        diag = g.c * dsum;
    } else {
        diag = g.c * (g.dim == 2 ? T(4) : T(6));
    }
    u[p] = f[p] / diag;
}

/* ------------------------------------------------------------------ */
/* Level hierarchy and the recursive V-cycle (Algorithm 1)              */
/* ------------------------------------------------------------------ */

/* Smoothers: red-black GS (red first in every sweep), omega-Jacobi, and the
 * symmetric red-black variant (red first before the coarse-grid correction,
 * black first after it). */
enum { SMOOTH_RBGS = 0, SMOOTH_JACOBI = 1, SMOOTH_RBGS_SYM = 2 };
/* Cycle types: V (one recursive call per level, Algorithm 1), W (two calls),
 * F (an F-cycle call followed by a V-cycle call). */
enum { CYCLE_V = 0, CYCLE_W = 1, CYCLE_F = 2 };

inline size_t npts(int dim, int n) { return dim == 3 ? (size_t)n * n * n : (size_t)n * n; }

/* constants of level with n nodes per axis, computed in double then rounded */
inline double level_c(int n) {
    const double h = 1.0 / (double)(n - 1);
    return 1.0 / (h * h);
}
inline double level_wd(int dim, int n, double omega) {
    const double h = 1.0 / (double)(n - 1);
    return (omega * (h * h)) / (2.0 * (double)dim);
}
/* constant stencil with centre entry s0: omega h^2 / s0 */
inline double level_wd_st(int n, double omega, double s0) {
    const double h = 1.0 / (double)(n - 1);
    return (omega * (h * h)) / s0;
}

template <typename S>
struct Hierarchy {
    typedef typename Arith<S>::type T;
    int dim, nlev, smoother, nu1, nu2;
    double omega;
    int cycle = CYCLE_V;   /* enum above */
    int coarse_n = 3;      /* edge of the coarsest level */
    int cg_iters = 0;      /* conjugate-gradient steps on a coarsest level with n > 3 */
    std::vector<int> n;               /* n[0] finest */
    std::vector<std::vector<S>> u, f;  /* iterate and right-hand side, storage type */
    std::vector<std::vector<T>> r, k;  /* residual and coefficient, arithmetic type */
    std::vector<T> st;                 /* constant stencil (same on every level), or empty */
    double st0 = 0.0;                  /* its centre entry as given */
    std::vector<S> tmp;

    Grid<S> grid(int l) const {
        Grid<S> g;
        g.dim = dim;
        g.n = n[(size_t)l];
        g.c = (T)level_c(g.n);
        g.wd = st.empty() ? (T)level_wd(dim, g.n, omega) : (T)level_wd_st(g.n, omega, st0);
        g.omega = (T)omega;
        g.k = k.empty() ? nullptr : k[(size_t)l].data();
        g.st = st.empty() ? nullptr : st.data();
        return g;
    }
    void set_stencil(const double* s64) {
        st.clear();
        if (!s64) return;
        for (int q = 0; q < 2 * dim + 1; ++q) st.push_back((T)s64[q]);
        st0 = s64[0];
    }
};

/* Build levels n, (n-1)/2+1, ..., 3.  Level 0 arrays u[0], f[0] are left
 * empty: the caller's arrays are used there.  k (if given) is converted to T
 * and injected to coarse levels. */
template <typename S>
void build(Hierarchy<S>& H, int dim, int n, const double* k64, int smoother, double omega, int nu1, int nu2,
           int coarse_n = 3) {
    typedef typename Arith<S>::type T;
    H.dim = dim;
    H.smoother = smoother;
    H.omega = omega;
    H.nu1 = nu1;
    H.nu2 = nu2;
    H.coarse_n = coarse_n < 3 ? 3 : coarse_n;
    H.n.clear();
    for (int m = n; m >= 3; m = (m - 1) / 2 + 1) {
        H.n.push_back(m);
        if (m <= H.coarse_n) break;
    }
    H.nlev = (int)H.n.size();
    H.u.assign((size_t)H.nlev, {});
    H.f.assign((size_t)H.nlev, {});
    H.r.assign((size_t)H.nlev, {});
    for (int l = 0; l < H.nlev; ++l) {
        const size_t sz = npts(dim, H.n[(size_t)l]);
        if (l > 0) {
            H.u[(size_t)l].assign(sz, T(0));
            H.f[(size_t)l].assign(sz, T(0));
        }
        H.r[(size_t)l].assign(sz, T(0));
    }
    H.k.clear();
    if (k64) {
        H.k.assign((size_t)H.nlev, {});
        H.k[0].resize(npts(dim, n));
        for (size_t p = 0; p < H.k[0].size(); ++p) H.k[0][p] = (T)k64[p];
        for (int l = 1; l < H.nlev; ++l) {
            const int nf = H.n[(size_t)l - 1], nc = H.n[(size_t)l];
            H.k[(size_t)l].resize(npts(dim, nc));
            const int K1 = dim == 3 ? nc : 1;
            for (int K = 0; K < K1; ++K)
                for (int J = 0; J < nc; ++J)
                    for (int I = 0; I < nc; ++I)
                        H.k[(size_t)l][(size_t)at(dim, nc, I, J, K)] =
                            H.k[(size_t)l - 1][(size_t)at(dim, nf, 2 * I, 2 * J, 2 * K)];
        }
    }
}

/* post = 1 for the smoothing sweeps after the coarse-grid correction */
template <typename S>
void smooth(Hierarchy<S>& H, int l, S* u, const S* f, int post = 0) {
    const Grid<S> g = H.grid(l);
    if (H.smoother == SMOOTH_RBGS)
        rbgs_sweep(g, u, f, 0);
    else if (H.smoother == SMOOTH_RBGS_SYM)
        rbgs_sweep(g, u, f, post);
    else
        jacobi_sweep(g, u, f, H.tmp);
}

/* <a, b> over inner nodes, products and sums in FP64: each x-row summed from
 * left to right, the row sums added in row order (k, then j) */
template <typename S>
double dot_inner(int dim, int n, const S* a, const S* b) {
    double s = 0.0;
    const int k0 = dim == 3 ? 1 : 0, k1 = dim == 3 ? n - 1 : 1;
    for (int k = k0; k < k1; ++k)
        for (int j = 1; j < n - 1; ++j) {
            double row = 0.0;
            for (int i = 1; i < n - 1; ++i) {
                const idx_t p = at(dim, n, i, j, k);
                row += (double)a[p] * (double)b[p];
            }
            s += row;
        }
    return s;
}

/* Coarsest level with more than one unknown: conjugate gradients (the
 * iterative option of Algorithm 1's coarsest-grid solve) on A u = f from
 * u = 0, a fixed number of steps (fewer only if the residual becomes exactly
 * zero).  Vectors in T; inner products in FP64, alpha and beta formed in
 * FP64 and rounded to T for the updates. */
template <typename S>
void coarsest_cg(const Grid<S>& g, S* u, const S* f, int iters) {
    typedef typename Arith<S>::type T;
    const int n = g.n, dim = g.dim;
    const size_t total = npts(dim, n);
    std::vector<S> r(total, T(0)), p(total, T(0)), q(total, T(0));
    const int k0 = dim == 3 ? 1 : 0, k1 = dim == 3 ? n - 1 : 1;
    for (size_t i = 0; i < total; ++i) u[i] = T(0);
    for (int k = k0; k < k1; ++k)
        for (int j = 1; j < n - 1; ++j)
            for (int i = 1; i < n - 1; ++i) {
                const idx_t x = at(dim, n, i, j, k);
                r[(size_t)x] = f[x];
                p[(size_t)x] = f[x];
            }
    double rr = dot_inner(dim, n, r.data(), r.data());
    for (int it = 0; it < iters && rr > 0.0; ++it) {
        for (int k = k0; k < k1; ++k)
            for (int j = 1; j < n - 1; ++j)
                for (int i = 1; i < n - 1; ++i) {
                    const idx_t x = at(dim, n, i, j, k);
                    if (g.st) {
                        q[(size_t)x] = apply_stencil(g, p.data(), x);
                    } else if (g.k) {
                        T dsum;
                        q[(size_t)x] = apply_varcoef(g, p.data(), x, &dsum);
                    } else {
                        q[(size_t)x] = apply_poisson(g, p.data(), x);
                    }
                }
        const double pq = dot_inner(dim, n, p.data(), q.data());
        if (!(pq > 0.0)) break;
        const T alpha = (T)(rr / pq);
        for (int k = k0; k < k1; ++k)
            for (int j = 1; j < n - 1; ++j)
                for (int i = 1; i < n - 1; ++i) {
                    const size_t x = (size_t)at(dim, n, i, j, k);
                    u[x] = u[x] + alpha * p[x];
                    r[x] = r[x] - alpha * q[x];
                }
        const double rr_new = dot_inner(dim, n, r.data(), r.data());
        const T beta = (T)(rr_new / rr);
        for (int k = k0; k < k1; ++k)
            for (int j = 1; j < n - 1; ++j)
                for (int i = 1; i < n - 1; ++i) {
                    const size_t x = (size_t)at(dim, n, i, j, k);
                    p[x] = r[x] + beta * p[x];
                }
        rr = rr_new;
    }
}

/* default number of conjugate-gradient steps on a coarsest level of edge n */
inline int cg_default_iters(int n) { return 4 * (n - 1); }

/* Multigrid cycle on level l (Algorithm 1 with gamma recursive calls):
 * kind V calls itself once, W twice, F an F-cycle then a V-cycle.  Each
 * call after the first continues from the coarse iterate the previous call
 * left (the zero guess precedes the first call only). */
template <typename S>
void mgcycle(Hierarchy<S>& H, int l, S* u, const S* f, int kind) {
    typedef typename Arith<S>::type T;
    const Grid<S> g = H.grid(l);
    if (l == H.nlev - 1) {
        if (g.n == 3)
            coarsest_solve(g, u, f);
        else
            coarsest_cg(g, u, f, H.cg_iters > 0 ? H.cg_iters : cg_default_iters(g.n));
        return;
    }
    for (int s = 0; s < H.nu1; ++s) smooth(H, l, u, f, 0);       /* presmoothing */
    T* r = H.r[(size_t)l].data();
    residual(g, u, f, r);                                         /* residual */
    S* fc = H.f[(size_t)l + 1].data();
    restrict_fw(H.dim, g.n, r, fc);                               /* restriction */
    S* uc = H.u[(size_t)l + 1].data();
    std::fill(H.u[(size_t)l + 1].begin(), H.u[(size_t)l + 1].end(), T(0)); /* zero guess */
    if (kind == CYCLE_V) {
        mgcycle(H, l + 1, uc, fc, CYCLE_V);                       /* recursion */
    } else if (kind == CYCLE_W) {
        mgcycle(H, l + 1, uc, fc, CYCLE_W);
        mgcycle(H, l + 1, uc, fc, CYCLE_W);
    } else {
        mgcycle(H, l + 1, uc, fc, CYCLE_F);
        mgcycle(H, l + 1, uc, fc, CYCLE_V);
    }
    prolong_correct(H.dim, g.n, u, uc);                           /* coarse-grid correction */
    for (int s = 0; s < H.nu2; ++s) smooth(H, l, u, f, 1);        /* postsmoothing */
}

/* Algorithm 1 on level l with solution u and right-hand side f */
template <typename S>
void vcycle(Hierarchy<S>& H, int l, S* u, const S* f) {
    mgcycle(H, l, u, f, H.cycle);
}

template <typename S>
Grid<S> make_grid(int dim, int n, const typename Arith<S>::type* kf, double omega) {
    typedef typename Arith<S>::type T;
    Grid<S> g;
    g.dim = dim;
    g.n = n;
    g.c = (T)level_c(n);
    g.wd = (T)level_wd(dim, n, omega);
    g.omega = (T)omega;
    g.k = kf;
    return g;
}

bool valid_edge(int n) { return n >= 3 && ((n - 1) & (n - 2)) == 0; }

/* ------------------------------------------------------------------ */
/* Cell-centred grids with a homogeneous Neumann boundary (Table 1's    */
/* cell-centred discretisation, Neumann boundary condition, constant    */
/* interpolation; the boundary of the paper's complex-diffusion         */
/* application, Section 4).  n = 2^L cells per axis, h = 1/n, cell        */
/* (i, j[, k]) centred at ((i+1/2)h, ...); values stored without ghost    */
/* cells, x fastest.  Zero flux across the boundary: a neighbour outside  */
/* the domain takes the cell's own value (ghost = mirror).  The operator  */
/* is singular (constants are in its kernel): the right-hand side is      */
/* projected onto mean zero and the iterate is kept at mean zero.         */
/* ------------------------------------------------------------------ */

inline idx_t cc_at(int dim, int n, int i, int j, int k) {
    return dim == 2 ? (idx_t)j * n + i : ((idx_t)k * n + j) * n + i;
}

/* number of faces of cell (i, j, k) on the boundary */
inline int cc_missing(int dim, int n, int i, int j, int k) {
    int m = (i == 0) + (i == n - 1) + (j == 0) + (j == n - 1);
    if (dim == 3) m += (k == 0) + (k == n - 1);
    return m;
}

/* (A u)_p = c (2d u_p - s), s the neighbour sum with ghost = own value,
 * summed as ((W+E)+(S+N))+(B+T) */
inline double cc_apply(int dim, int n, double c, const double* u, int i, int j, int k) {
    const idx_t p = cc_at(dim, n, i, j, k);
    const double uC = u[p];
    const double uW = i > 0 ? u[p - 1] : uC, uE = i < n - 1 ? u[p + 1] : uC;
    const double uS = j > 0 ? u[p - n] : uC, uN = j < n - 1 ? u[p + n] : uC;
    if (dim == 2) return c * (4.0 * uC - ((uW + uE) + (uS + uN)));
    const idx_t sz = (idx_t)n * n;
    const double uB = k > 0 ? u[p - sz] : uC, uT = k < n - 1 ? u[p + sz] : uC;
    return c * (6.0 * uC - (((uW + uE) + (uS + uN)) + (uB + uT)));
}

/* per-level constants: c = 1/h^2, wd[m] = omega h^2 / (2d - m): omega times
 * the inverse of the true diagonal c (2d - m) of a cell with m boundary
 * faces (m <= d) */
struct CCLevel {
    int dim, n;
    double c, wd[4];
};
inline CCLevel cc_level(int dim, int n, double omega) {
    CCLevel L;
    L.dim = dim;
    L.n = n;
    const double h = 1.0 / (double)n;
    L.c = 1.0 / (h * h);
    for (int m = 0; m < 4; ++m) L.wd[m] = (omega * (h * h)) / (double)(2 * dim - m);
    return L;
}

inline int cc_k1(int dim, int n) { return dim == 3 ? n : 1; }

/* relaxation u + omega diag^-1 (f - A u) at one cell */
inline double cc_relax(const CCLevel& L, const double* u, const double* f, int i, int j, int k) {
    const idx_t p = cc_at(L.dim, L.n, i, j, k);
    const double r = f[p] - cc_apply(L.dim, L.n, L.c, u, i, j, k);
    return u[p] + L.wd[cc_missing(L.dim, L.n, i, j, k)] * r;
}

void cc_rbgs(const CCLevel& L, double* u, const double* f) {
    const int n = L.n;
    for (int colour = 0; colour < 2; ++colour)
        for (int k = 0; k < cc_k1(L.dim, n); ++k)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i)
                    if (((i + j + k) & 1) == colour) u[cc_at(L.dim, n, i, j, k)] = cc_relax(L, u, f, i, j, k);
}

void cc_jacobi(const CCLevel& L, double* u, const double* f, std::vector<double>& tmp) {
    const int n = L.n;
    const size_t N = L.dim == 3 ? (size_t)n * n * n : (size_t)n * n;
    tmp.assign(u, u + N);
    for (int k = 0; k < cc_k1(L.dim, n); ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) tmp[(size_t)cc_at(L.dim, n, i, j, k)] = cc_relax(L, u, f, i, j, k);
    std::memcpy(u, tmp.data(), N * sizeof(double));
}

void cc_residual(const CCLevel& L, const double* u, const double* f, double* r) {
    const int n = L.n;
    for (int k = 0; k < cc_k1(L.dim, n); ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                const idx_t p = cc_at(L.dim, n, i, j, k);
                r[p] = f[p] - cc_apply(L.dim, n, L.c, u, i, j, k);
            }
}

/* coarse cell = average of its 2^d children (cell-centred restriction) */
void cc_restrict(int dim, int nf, const double* r, double* fc) {
    const int nc = nf / 2;
    for (int K = 0; K < cc_k1(dim, nc); ++K)
        for (int J = 0; J < nc; ++J)
            for (int I = 0; I < nc; ++I) {
                const int i = 2 * I, j = 2 * J, k = 2 * K;
                const double q0 = (r[cc_at(dim, nf, i, j, k)] + r[cc_at(dim, nf, i + 1, j, k)]) +
                                  (r[cc_at(dim, nf, i, j + 1, k)] + r[cc_at(dim, nf, i + 1, j + 1, k)]);
                if (dim == 2) {
                    fc[cc_at(dim, nc, I, J, K)] = 0.25 * q0;
                } else {
                    const double q1 = (r[cc_at(dim, nf, i, j, k + 1)] + r[cc_at(dim, nf, i + 1, j, k + 1)]) +
                                      (r[cc_at(dim, nf, i, j + 1, k + 1)] + r[cc_at(dim, nf, i + 1, j + 1, k + 1)]);
                    fc[cc_at(dim, nc, I, J, K)] = 0.125 * (q0 + q1);
                }
            }
}

/* constant interpolation and correction: each fine cell gets its parent's value */
void cc_prolong_correct(int dim, int nf, double* u, const double* ec) {
    const int nc = nf / 2;
    for (int k = 0; k < cc_k1(dim, nf); ++k)
        for (int j = 0; j < nf; ++j)
            for (int i = 0; i < nf; ++i) {
                const idx_t p = cc_at(dim, nf, i, j, k);
                u[p] = u[p] + ec[cc_at(dim, nc, i / 2, j / 2, dim == 3 ? k / 2 : 0)];
            }
}

/* sum of all cells: each x-row left to right, the rows of a plane in order,
 * the planes in order */
double cc_sum(int dim, int n, const double* u) {
    double total = 0.0;
    for (int k = 0; k < cc_k1(dim, n); ++k) {
        double plane = 0.0;
        for (int j = 0; j < n; ++j) {
            double row = 0.0;
            for (int i = 0; i < n; ++i) row += u[cc_at(dim, n, i, j, k)];
            plane += row;
        }
        total += plane;
    }
    return total;
}

inline size_t cc_cells(int dim, int n) { return dim == 3 ? (size_t)n * n * n : (size_t)n * n; }

/* v -= mean(v) (mean = sum / number of cells) */
void cc_remove_mean(int dim, int n, double* v) {
    const size_t N = cc_cells(dim, n);
    const double mean = cc_sum(dim, n, v) / (double)N;
    for (size_t p = 0; p < N; ++p) v[p] = v[p] - mean;
}

/* ||f - A u||_2 over all cells, squares summed per x-row, then the rows of a
 * plane, then the planes (partial sums keep the rounding of the sum small) */
double cc_residual_norm(const CCLevel& L, const double* u, const double* f) {
    const int n = L.n;
    double s = 0.0;
    for (int k = 0; k < cc_k1(L.dim, n); ++k) {
        double plane = 0.0;
        for (int j = 0; j < n; ++j) {
            double row = 0.0;
            for (int i = 0; i < n; ++i) {
                const double r = f[cc_at(L.dim, n, i, j, k)] - cc_apply(L.dim, n, L.c, u, i, j, k);
                row += r * r;
            }
            plane += row;
        }
        s += plane;
    }
    return std::sqrt(s);
}

struct CCHierarchy {
    int dim, nlev, smoother, nu1, nu2, cycle;
    double omega;
    std::vector<int> n;
    std::vector<std::vector<double>> u, f, r;
    std::vector<double> tmp;
};

void cc_build(CCHierarchy& H, int dim, int n, int smoother, double omega, int nu1, int nu2, int cycle) {
    H.dim = dim;
    H.smoother = smoother;
    H.omega = omega;
    H.nu1 = nu1;
    H.nu2 = nu2;
    H.cycle = cycle;
    H.n.clear();
    for (int m = n; m >= 1; m /= 2) H.n.push_back(m);
    H.nlev = (int)H.n.size();
    H.u.assign((size_t)H.nlev, {});
    H.f.assign((size_t)H.nlev, {});
    H.r.assign((size_t)H.nlev, {});
    for (int l = 0; l < H.nlev; ++l) {
        const size_t N = cc_cells(dim, H.n[(size_t)l]);
        if (l > 0) {
            H.u[(size_t)l].assign(N, 0.0);
            H.f[(size_t)l].assign(N, 0.0);
        }
        H.r[(size_t)l].assign(N, 0.0);
    }
}

void cc_smooth(CCHierarchy& H, const CCLevel& L, double* u, const double* f) {
    if (H.smoother == SMOOTH_JACOBI) cc_jacobi(L, u, f, H.tmp);
    else cc_rbgs(L, u, f);
}

/* Algorithm 1 on a cell-centred level; the coarsest level is a single cell,
 * whose operator is zero: its correction is 0 (the constant is fixed by the
 * mean-zero condition). */
void cc_cycle(CCHierarchy& H, int l, double* u, const double* f, int kind) {
    const int n = H.n[(size_t)l];
    if (l == H.nlev - 1) {
        for (size_t p = 0; p < cc_cells(H.dim, n); ++p) u[p] = 0.0;
        return;
    }
    const CCLevel L = cc_level(H.dim, n, H.omega);
    for (int s = 0; s < H.nu1; ++s) cc_smooth(H, L, u, f);
    double* r = H.r[(size_t)l].data();
    cc_residual(L, u, f, r);
    double* fc = H.f[(size_t)l + 1].data();
    cc_restrict(H.dim, n, r, fc);
    double* uc = H.u[(size_t)l + 1].data();
    std::fill(H.u[(size_t)l + 1].begin(), H.u[(size_t)l + 1].end(), 0.0);
    if (kind == CYCLE_V) {
        cc_cycle(H, l + 1, uc, fc, CYCLE_V);
    } else if (kind == CYCLE_W) {
        cc_cycle(H, l + 1, uc, fc, CYCLE_W);
        cc_cycle(H, l + 1, uc, fc, CYCLE_W);
    } else {
        cc_cycle(H, l + 1, uc, fc, CYCLE_F);
        cc_cycle(H, l + 1, uc, fc, CYCLE_V);
    }
    cc_prolong_correct(H.dim, n, u, uc);
    for (int s = 0; s < H.nu2; ++s) cc_smooth(H, L, u, f);
}

bool cc_valid(int dim, int n) { return (dim == 2 || dim == 3) && n >= 2 && (n & (n - 1)) == 0; }

/* ------------------------------------------------------------------ */
/* Complex diffusion (Section 4, Eq. (2)): u_t = div(g(Im u) grad u) on   */
/* the unit square / cube with a homogeneous Neumann boundary,            */
/* g(s) = e^{i theta} / (1 + (s / (k theta))^2).  Cell-centred averaged   */
/* finite differences (face diffusivity = mean of the two cells' values), */
/* implicit Euler in time, and per time step the full approximation       */
/* scheme (FAS) with lagged diffusivity: every smoothing sweep and every  */
/* residual uses g of the iterate it starts from.  Transfers: averaging   */
/* restriction, constant interpolation.  Complex values are (re, im)      */
/* pairs of doubles with the arithmetic written out in a fixed order.     */
/* ------------------------------------------------------------------ */

struct Cx {
    double re, im;
};
inline Cx cx_add(Cx a, Cx b) { return Cx{a.re + b.re, a.im + b.im}; }
inline Cx cx_sub(Cx a, Cx b) { return Cx{a.re - b.re, a.im - b.im}; }
inline Cx cx_mul(Cx a, Cx b) { return Cx{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
inline Cx cx_div(Cx a, Cx b) {
    const double den = b.re * b.re + b.im * b.im;
    return Cx{(a.re * b.re + a.im * b.im) / den, (a.im * b.re - a.re * b.im) / den};
}
inline Cx cx_scale(double s, Cx a) { return Cx{s * a.re, s * a.im}; }

/* parameters of the complex-diffusion problem; ct, st = cos theta, sin theta */
struct CDParams {
    int dim;
    double tau, itau, ktheta, ct, st;
};

/* g(Im u) = (cos theta, sin theta) / (1 + (Im u / (k theta))^2) */
inline Cx cd_g(const CDParams& P, Cx u) {
    const double s = u.im / P.ktheta;
    const double q = 1.0 / (1.0 + s * s);
    return Cx{P.ct * q, P.st * q};
}

/* flux sum F = sum over faces of g_face (u_q - u_p) and diagonal sum S of the
 * face coefficients, faces W, E, S, N[, B, T] paired as ((W+E)+(S+N))+(B+T);
 * a face on the boundary carries no flux (its terms are 0) */
inline void cd_faces(int dim, int n, const Cx* u, const Cx* g, int i, int j, int k, Cx* F, Cx* S) {
    const idx_t p = cc_at(dim, n, i, j, k);
    const idx_t sz = (idx_t)n * n;
    const Cx zero{0.0, 0.0};
    const Cx up = u[p], gp = g[p];
    auto face = [&](bool inside, idx_t q, Cx* t, Cx* gf) {
        if (!inside) {
            *t = zero;
            *gf = zero;
            return;
        }
        const Cx gq = g[q];
        *gf = Cx{0.5 * (gp.re + gq.re), 0.5 * (gp.im + gq.im)};
        *t = cx_mul(*gf, cx_sub(u[q], up));
    };
    Cx tW, tE, tS, tN, gW, gE, gS, gN;
    face(i > 0, p - 1, &tW, &gW);
    face(i < n - 1, p + 1, &tE, &gE);
    face(j > 0, p - n, &tS, &gS);
    face(j < n - 1, p + n, &tN, &gN);
    Cx f2 = cx_add(cx_add(tW, tE), cx_add(tS, tN));
    Cx s2 = cx_add(cx_add(gW, gE), cx_add(gS, gN));
    if (dim == 3) {
        Cx tB, tT, gB, gT;
        face(k > 0, p - sz, &tB, &gB);
        face(k < n - 1, p + sz, &tT, &gT);
        f2 = cx_add(f2, cx_add(tB, tT));
        s2 = cx_add(s2, cx_add(gB, gT));
    }
    *F = f2;
    *S = s2;
}

/* N(u)_p = u_p / tau - c F (the implicit-Euler operator with diffusivity g) */
inline Cx cd_apply(const CDParams& P, int n, double c, const Cx* u, const Cx* g, int i, int j, int k) {
    Cx F, S;
    cd_faces(P.dim, n, u, g, i, j, k, &F, &S);
    const Cx up = u[cc_at(P.dim, n, i, j, k)];
    return Cx{P.itau * up.re - c * F.re, P.itau * up.im - c * F.im};
}

void cd_compute_g(const CDParams& P, int n, const Cx* u, Cx* g) {
    const size_t N = cc_cells(P.dim, n);
    for (size_t p = 0; p < N; ++p) g[p] = cd_g(P, u[p]);
}

/* one smoothing sweep with the diffusivity frozen at the iterate the sweep
 * starts from: RBGS (red cells, then black, in place) or Jacobi (out of place);
 * update u + omega r / D with D = 1/tau + c S the diagonal */
void cd_sweep(const CDParams& P, int n, double c, int smoother, double omega, Cx* u, const Cx* f,
              std::vector<Cx>& g, std::vector<Cx>& tmp) {
    const int dim = P.dim;
    const size_t N = cc_cells(dim, n);
    g.resize(N);
    cd_compute_g(P, n, u, g.data());
    auto relax = [&](const Cx* src, int i, int j, int k) {
        const idx_t p = cc_at(dim, n, i, j, k);
        Cx F, S;
        cd_faces(dim, n, src, g.data(), i, j, k, &F, &S);
        const Cx up = src[p];
        const Cx Nu{P.itau * up.re - c * F.re, P.itau * up.im - c * F.im};
        const Cx r = cx_sub(f[p], Nu);
        const Cx D{P.itau + c * S.re, c * S.im};
        return cx_add(up, cx_scale(omega, cx_div(r, D)));
    };
    if (smoother == SMOOTH_JACOBI) {
        tmp.assign(u, u + N);
        for (int k = 0; k < cc_k1(dim, n); ++k)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i) tmp[(size_t)cc_at(dim, n, i, j, k)] = relax(u, i, j, k);
        std::memcpy(u, tmp.data(), N * sizeof(Cx));
        return;
    }
    for (int colour = 0; colour < 2; ++colour)
        for (int k = 0; k < cc_k1(dim, n); ++k)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i)
                    if (((i + j + k) & 1) == colour) u[cc_at(dim, n, i, j, k)] = relax(u, i, j, k);
}

/* r = f - N(u) with g of u */
void cd_residual(const CDParams& P, int n, double c, const Cx* u, const Cx* f, std::vector<Cx>& g, Cx* r) {
    const size_t N = cc_cells(P.dim, n);
    g.resize(N);
    cd_compute_g(P, n, u, g.data());
    for (int k = 0; k < cc_k1(P.dim, n); ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                const idx_t p = cc_at(P.dim, n, i, j, k);
                r[p] = cx_sub(f[p], cd_apply(P, n, c, u, g.data(), i, j, k));
            }
}

/* average of the 2^d children, componentwise (as cc_restrict) */
void cd_average(int dim, int nf, const Cx* a, Cx* out) {
    const int nc = nf / 2;
    const size_t Nf = cc_cells(dim, nf), Nc = cc_cells(dim, nc);
    std::vector<double> re(Nf), im(Nf), cre(Nc), cim(Nc);
    for (size_t p = 0; p < Nf; ++p) {
        re[p] = a[p].re;
        im[p] = a[p].im;
    }
    cc_restrict(dim, nf, re.data(), cre.data());
    cc_restrict(dim, nf, im.data(), cim.data());
    for (size_t q = 0; q < Nc; ++q) out[q] = Cx{cre[q], cim[q]};
}

/* ||r||_2 with |r_p|^2 = re^2 + im^2, summed per x-row, plane, all */
double cd_norm(int dim, int n, const Cx* r) {
    double s = 0.0;
    for (int k = 0; k < cc_k1(dim, n); ++k) {
        double plane = 0.0;
        for (int j = 0; j < n; ++j) {
            double row = 0.0;
            for (int i = 0; i < n; ++i) {
                const Cx v = r[cc_at(dim, n, i, j, k)];
                row += v.re * v.re + v.im * v.im;
            }
            plane += row;
        }
        s += plane;
    }
    return std::sqrt(s);
}

struct CDHierarchy {
    CDParams P;
    int nlev, smoother, nu1, nu2;
    double omega;
    std::vector<int> n;
    std::vector<std::vector<Cx>> u, f, uh, r;
    std::vector<Cx> g, tmp;
};

void cd_build(CDHierarchy& H, const CDParams& P, int n, int smoother, double omega, int nu1, int nu2) {
    H.P = P;
    H.smoother = smoother;
    H.omega = omega;
    H.nu1 = nu1;
    H.nu2 = nu2;
    H.n.clear();
    for (int m = n; m >= 1; m /= 2) H.n.push_back(m);
    H.nlev = (int)H.n.size();
    H.u.assign((size_t)H.nlev, {});
    H.f.assign((size_t)H.nlev, {});
    H.uh.assign((size_t)H.nlev, {});
    H.r.assign((size_t)H.nlev, {});
    for (int l = 0; l < H.nlev; ++l) {
        const size_t N = cc_cells(P.dim, H.n[(size_t)l]);
        H.r[(size_t)l].assign(N, Cx{0.0, 0.0});
        if (l > 0) {
            H.u[(size_t)l].assign(N, Cx{0.0, 0.0});
            H.f[(size_t)l].assign(N, Cx{0.0, 0.0});
            H.uh[(size_t)l].assign(N, Cx{0.0, 0.0});
        }
    }
}

inline double cd_c(int n) {
    const double h = 1.0 / (double)n;
    return 1.0 / (h * h);
}

/* One FAS V-cycle on level l for N(u) = f (the coarse problem of level l+1
 * is N_c(u_c) = N_c(R u) + R (f - N(u)) from u_c = R u; the correction
 * u_c - R u is interpolated back).  Coarsest level (one cell): N(u) = u/tau,
 * solved exactly: u = tau f. */
void cd_fas(CDHierarchy& H, int l, Cx* u, const Cx* f) {
    const CDParams& P = H.P;
    const int n = H.n[(size_t)l];
    const double c = cd_c(n);
    if (l == H.nlev - 1) {
        for (size_t p = 0; p < cc_cells(P.dim, n); ++p) u[p] = cx_scale(P.tau, f[p]);
        return;
    }
    for (int s = 0; s < H.nu1; ++s) cd_sweep(P, n, c, H.smoother, H.omega, u, f, H.g, H.tmp);
    Cx* r = H.r[(size_t)l].data();
    cd_residual(P, n, c, u, f, H.g, r);
    const int nc = H.n[(size_t)l + 1];
    const size_t Nc = cc_cells(P.dim, nc);
    Cx* uh = H.uh[(size_t)l + 1].data();
    Cx* fc = H.f[(size_t)l + 1].data();
    Cx* uc = H.u[(size_t)l + 1].data();
    cd_average(P.dim, n, u, uh);
    std::vector<Cx> rc(Nc);
    cd_average(P.dim, n, r, rc.data());
    /* fc = N_c(uh) + R r, with g of uh */
    std::vector<Cx> gc(Nc);
    cd_compute_g(P, nc, uh, gc.data());
    const double cc = cd_c(nc);
    for (int k = 0; k < cc_k1(P.dim, nc); ++k)
        for (int j = 0; j < nc; ++j)
            for (int i = 0; i < nc; ++i) {
                const idx_t q = cc_at(P.dim, nc, i, j, k);
                fc[q] = cx_add(cd_apply(P, nc, cc, uh, gc.data(), i, j, k), rc[(size_t)q]);
            }
    for (size_t q = 0; q < Nc; ++q) uc[q] = uh[q];
    cd_fas(H, l + 1, uc, fc);
    /* u += P (u_c - uh) (constant interpolation of the coarse correction) */
    for (int k = 0; k < cc_k1(P.dim, n); ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                const idx_t p = cc_at(P.dim, n, i, j, k);
                const idx_t q = cc_at(P.dim, nc, i / 2, j / 2, P.dim == 3 ? k / 2 : 0);
                u[p] = cx_add(u[p], cx_sub(uc[q], uh[q]));
            }
    for (int s = 0; s < H.nu2; ++s) cd_sweep(P, n, c, H.smoother, H.omega, u, f, H.g, H.tmp);
}

CDParams cd_params(int dim, double tau, double theta, double k, double ct, double st) {
    CDParams P;
    P.dim = dim;
    P.tau = tau;
    P.itau = 1.0 / tau;
    P.ktheta = k * theta;
    P.ct = ct;
    P.st = st;
    return P;
}

} /* namespace */

/* ==================================================================== */
/* C interface (called through ctypes by the tests).                      */
/* Every array is dense, x fastest, n nodes per axis, boundary included. */
/* Return codes: 0 ok, 1 not converged within max_cycles, -1 bad args.    */
/* ==================================================================== */

extern "C" {

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}



/* r = f - A u (inner), 0 on boundary */
void orc_residual_f64(int dim, int n, const double* k, const double* u, const double* f, double* r) {
    const Grid<double> g = make_grid<double>(dim, n, k, 1.0);
    residual(g, u, f, r);
}
void orc_residual_f32(int dim, int n, const float* k, const float* u, const float* f, float* r) {
    const Grid<float> g = make_grid<float>(dim, n, k, 1.0);
    residual(g, u, f, r);
}

/* one smoothing sweep in place (smoother 0 = RBGS red first, 1 = Jacobi,
 * 2 = RBGS black first: the post-smoothing sweep of the symmetric variant) */
void orc_smooth_f64(int dim, int n, const double* k, int smoother, double omega, double* u, const double* f) {
    const Grid<double> g = make_grid<double>(dim, n, k, omega);
    std::vector<double> tmp;
    if (smoother == SMOOTH_JACOBI) jacobi_sweep(g, u, f, tmp);
    else rbgs_sweep(g, u, f, smoother == SMOOTH_RBGS_SYM ? 1 : 0);
}
void orc_smooth_f32(int dim, int n, const float* k, int smoother, double omega, float* u, const float* f) {
    const Grid<float> g = make_grid<float>(dim, n, k, omega);
    std::vector<float> tmp;
    if (smoother == SMOOTH_JACOBI) jacobi_sweep(g, u, f, tmp);
    else rbgs_sweep(g, u, f, smoother == SMOOTH_RBGS_SYM ? 1 : 0);
}

/* Coarsest-level conjugate gradients alone (n >= 3), iters steps (0: default 4(n-1)). */
void orc_coarsest_cg_f64(int dim, int n, const double* k, int iters, double* u, const double* f) {
    const Grid<double> g = make_grid<double>(dim, n, k, 1.0);
    coarsest_cg(g, u, f, iters > 0 ? iters : cg_default_iters(n));
}
void orc_coarsest_cg_f32(int dim, int n, const float* k, int iters, float* u, const float* f) {
    const Grid<float> g = make_grid<float>(dim, n, k, 1.0);
    coarsest_cg(g, u, f, iters > 0 ? iters : cg_default_iters(n));
}

/* only the red (colour 0) or black (colour 1) half of an RBGS sweep */
void orc_rbgs_colour_f64(int dim, int n, const double* k, double omega, int colour, int reverse, double* u,
                         const double* f) {
    const Grid<double> g = make_grid<double>(dim, n, k, omega);
    const int k0 = dim == 3 ? 1 : 0, k1 = dim == 3 ? n - 1 : 1;
    /* serial loops, optionally in reversed lexicographic order */
    for (int kk = 0; kk < k1 - k0; ++kk)
        for (int jj = 1; jj < n - 1; ++jj)
            for (int ii = 1; ii < n - 1; ++ii) {
                const int k = reverse ? k1 - 1 - kk : k0 + kk;
                const int j = reverse ? n - 1 - jj : jj;
                const int i = reverse ? n - 1 - ii : ii;
                const int kc = dim == 3 ? k : 0;
                if (((i + j + kc) & 1) != colour) continue;
                const idx_t p = at(dim, n, i, j, k);
                u[p] = smooth_at(g, u, f, p);
            }
}

void orc_restrict_f64(int dim, int nf, const double* r, double* fc) { restrict_fw(dim, nf, r, fc); }
void orc_restrict_f32(int dim, int nf, const float* r, float* fc) { restrict_fw(dim, nf, r, fc); }

void orc_prolong_correct_f64(int dim, int nf, double* u, const double* ec) { prolong_correct(dim, nf, u, ec); }
void orc_prolong_correct_f32(int dim, int nf, float* u, const float* ec) { prolong_correct(dim, nf, u, ec); }

void orc_coarsest_f64(int dim, const double* k, double* u, const double* f) {
    const Grid<double> g = make_grid<double>(dim, 3, k, 1.0);
    coarsest_solve(g, u, f);
}

double orc_residual_norm_f64(int dim, int n, const double* k, const double* u, const double* f) {
    const Grid<double> g = make_grid<double>(dim, n, k, 1.0);
    return residual_norm(g, u, f);
}

/* Cycle options beyond Algorithm 1's V-cycle with an exact 3-point coarsest
 * solve: cycle type (0 V, 1 W, 2 F), edge of the coarsest level (3 = one
 * unknown, solved exactly; larger: conjugate gradients, cg_iters steps, 0 =
 * default). */
static bool valid_opts(int n, int cycle, int coarse_n) {
    return cycle >= CYCLE_V && cycle <= CYCLE_F && valid_edge(coarse_n) && coarse_n <= n;
}

/* One multigrid cycle on the finest grid, u updated in place. */
int orc_cycle_f64(int dim, int n, const double* k, int smoother, double omega, int nu1, int nu2, int cycle,
                  int coarse_n, int cg_iters, double* u, const double* f) {
    if ((dim != 2 && dim != 3) || !valid_edge(n) || !valid_opts(n, cycle, coarse_n)) return -1;
    Hierarchy<double> H;
    build(H, dim, n, k, smoother, omega, nu1, nu2, coarse_n);
    H.cycle = cycle;
    H.cg_iters = cg_iters;
    vcycle(H, 0, u, f);
    return 0;
}

/* Same cycle in single precision (u, f, k in float). */
int orc_cycle_f32(int dim, int n, const float* k32, int smoother, double omega, int nu1, int nu2, int cycle,
                  int coarse_n, int cg_iters, float* u, const float* f) {
    if ((dim != 2 && dim != 3) || !valid_edge(n) || !valid_opts(n, cycle, coarse_n)) return -1;
    Hierarchy<float> H;
    std::vector<double> k64;
    if (k32) k64.assign(k32, k32 + npts(dim, n));
    build(H, dim, n, k32 ? k64.data() : nullptr, smoother, omega, nu1, nu2, coarse_n);
    H.cycle = cycle;
    H.cg_iters = cg_iters;
    vcycle(H, 0, u, f);
    return 0;
}

/* One V(nu1,nu2) cycle on the finest grid, u updated in place. */
int orc_vcycle_f64(int dim, int n, const double* k, int smoother, double omega, int nu1, int nu2, double* u,
                   const double* f) {
    return orc_cycle_f64(dim, n, k, smoother, omega, nu1, nu2, CYCLE_V, 3, 0, u, f);
}

/* Same cycle in single precision (u, f, k in float). */
int orc_vcycle_f32(int dim, int n, const float* k32, int smoother, double omega, int nu1, int nu2, float* u,
                   const float* f) {
    return orc_cycle_f32(dim, n, k32, smoother, omega, nu1, nu2, CYCLE_V, 3, 0, u, f);
}

/* Solve loop of the Layer-4 Application function: rho_0 = ||f - A u||, then
 * cycles until rho_k <= tol * rho_0 or max_cycles.  hist (len max_cycles+1,
 * may be NULL) receives rho_0..rho_k; *cycles the number of cycles done. */
int orc_solve_mg_f64(int dim, int n, const double* k, int smoother, double omega, int nu1, int nu2, int cycle,
                     int coarse_n, int cg_iters, double* u, const double* f, double tol, int max_cycles,
                     double* hist, int* cycles) {
    if ((dim != 2 && dim != 3) || !valid_edge(n) || max_cycles < 0 || !valid_opts(n, cycle, coarse_n)) return -1;
    Hierarchy<double> H;
    build(H, dim, n, k, smoother, omega, nu1, nu2, coarse_n);
    H.cycle = cycle;
    H.cg_iters = cg_iters;
    const Grid<double> g0 = H.grid(0);
    const double rho0 = residual_norm(g0, u, f);
    if (hist) hist[0] = rho0;
    int it = 0;
    int status = 1;
    if (rho0 == 0.0) status = 0;
    while (status == 1 && it < max_cycles) {
        vcycle(H, 0, u, f);
        ++it;
        const double rho = residual_norm(g0, u, f);
        if (hist) hist[it] = rho;
        if (rho <= tol * rho0) status = 0;
    }
    if (cycles) *cycles = it;
    return status;
}

int orc_solve_f64(int dim, int n, const double* k, int smoother, double omega, int nu1, int nu2, double* u,
                  const double* f, double tol, int max_cycles, double* hist, int* cycles) {
    return orc_solve_mg_f64(dim, n, k, smoother, omega, nu1, nu2, CYCLE_V, 3, 0, u, f, tol, max_cycles, hist,
                            cycles);
}

/* ------------------------------------------------------------------ */
/* Constant stencil (FP64): st holds 2d+1 coefficients, centre first,    */
/* then -x, +x, -y, +y[, -z, +z]; A = (1/h^2) stencil on every level.     */
/* ------------------------------------------------------------------ */

static Grid<double> st_grid(int dim, int n, const double* st, double omega) {
    Grid<double> g = make_grid<double>(dim, n, nullptr, omega);
    g.st = st;
    g.wd = level_wd_st(n, omega, st[0]);
    return g;
}
void orc_st_residual(int dim, int n, const double* st, const double* u, const double* f, double* r) {
    residual(st_grid(dim, n, st, 1.0), u, f, r);
}
/* one sweep in place: smoother 0 RBGS red first, 1 Jacobi, 2 RBGS black first */
void orc_st_smooth(int dim, int n, const double* st, int smoother, double omega, double* u, const double* f) {
    const Grid<double> g = st_grid(dim, n, st, omega);
    std::vector<double> tmp;
    if (smoother == SMOOTH_JACOBI) jacobi_sweep(g, u, f, tmp);
    else rbgs_sweep(g, u, f, smoother == SMOOTH_RBGS_SYM ? 1 : 0);
}
void orc_st_coarsest(int dim, const double* st, double* u, const double* f) {
    coarsest_solve(st_grid(dim, 3, st, 1.0), u, f);
}
double orc_st_residual_norm(int dim, int n, const double* st, const double* u, const double* f) {
    return residual_norm(st_grid(dim, n, st, 1.0), u, f);
}
/* cycles (V 0, W 1, F 2) down to n = 3 until ||f - A u|| <= tol rho_0 or
 * max_cycles, as orc_solve_mg_f64 */
int orc_st_solve(int dim, int n, const double* st, int smoother, double omega, int nu1, int nu2, int cycle,
                 double* u, const double* f, double tol, int max_cycles, double* hist, int* cycles) {
    if ((dim != 2 && dim != 3) || !valid_edge(n) || max_cycles < 0 || !valid_opts(n, cycle, 3) || !st ||
        !(st[0] > 0.0))
        return -1;
    Hierarchy<double> H;
    build(H, dim, n, nullptr, smoother, omega, nu1, nu2, 3);
    H.set_stencil(st);
    H.cycle = cycle;
    const Grid<double> g0 = H.grid(0);
    const double rho0 = residual_norm(g0, u, f);
    if (hist) hist[0] = rho0;
    int it = 0;
    int status = rho0 == 0.0 ? 0 : 1;
    while (status == 1 && it < max_cycles) {
        vcycle(H, 0, u, f);
        ++it;
        const double rho = residual_norm(g0, u, f);
        if (hist) hist[it] = rho;
        if (rho <= tol * rho0) status = 0;
    }
    if (cycles) *cycles = it;
    return status;
}

/* One FP64 refinement pass: u += e (inner nodes), r = f - A u in FP64,
 * r32 = (float) r, returns ||r||_2.  k64 may be NULL. */
double orc_ir_update_f32(int dim, int n, const double* k64, double* u, const float* e, const double* f, float* r32) {
    const Grid<double> g = make_grid<double>(dim, n, k64, 1.0);
    const size_t total = npts(dim, n);
    const int k0 = dim == 3 ? 1 : 0, k1 = dim == 3 ? n - 1 : 1;
    for (int k = k0; k < k1; ++k)
        for (int j = 1; j < n - 1; ++j)
            for (int i = 1; i < n - 1; ++i) {
                const idx_t p = at(dim, n, i, j, k);
                u[p] = u[p] + (double)e[p];
            }
    std::vector<double> r(total);
    residual(g, u, f, r.data());
    for (size_t p = 0; p < total; ++p) r32[p] = (float)r[p];
    return residual_norm(g, u, f);
}

/* Mixed precision: single-precision cycles on the correction equation
 * A e = r inside FP64 iterative refinement.  Each outer step: u += e, r = f -
 * A u and ||r|| in FP64, r rounded to float, then one float cycle from
 * e = 0.  hist[0..] holds the FP64 residual norms; stop as in orc_solve_f64. */
int orc_solve_ir_mg_f32(int dim, int n, const double* k64, int smoother, double omega, int nu1, int nu2, int cycle,
                        int coarse_n, int cg_iters, double* u, const double* f, double tol, int max_cycles,
                        double* hist, int* cycles) {
    if ((dim != 2 && dim != 3) || !valid_edge(n) || max_cycles < 0 || !valid_opts(n, cycle, coarse_n)) return -1;
    Hierarchy<float> H;
    build(H, dim, n, k64, smoother, omega, nu1, nu2, coarse_n);
    H.cycle = cycle;
    H.cg_iters = cg_iters;
    const size_t total = npts(dim, n);
    std::vector<float> e(total, 0.0f), r32(total, 0.0f);
    double rho0 = orc_ir_update_f32(dim, n, k64, u, e.data(), f, r32.data());
    if (hist) hist[0] = rho0;
    int it = 0;
    int status = rho0 == 0.0 ? 0 : 1;
    while (status == 1 && it < max_cycles) {
        std::fill(e.begin(), e.end(), 0.0f);
        vcycle(H, 0, e.data(), r32.data());
        ++it;
        const double rho = orc_ir_update_f32(dim, n, k64, u, e.data(), f, r32.data());
        if (hist) hist[it] = rho;
        if (rho <= tol * rho0) status = 0;
    }
    if (cycles) *cycles = it;
    return status;
}

int orc_solve_ir_f32(int dim, int n, const double* k64, int smoother, double omega, int nu1, int nu2, double* u,
                     const double* f, double tol, int max_cycles, double* hist, int* cycles) {
    return orc_solve_ir_mg_f32(dim, n, k64, smoother, omega, nu1, nu2, CYCLE_V, 3, 0, u, f, tol, max_cycles, hist,
                               cycles);
}

/* ------------------------------------------------------------------ */
/* Half-precision storage form of the refinement (FP16 cells, float     */
/* arithmetic, FP64 outer residual).  Arrays of binary16 cells are passed */
/* as their 16-bit patterns.                                             */
/* ------------------------------------------------------------------ */

void orc_half_from_float(const float* x, uint16_t* out, long long count) {
    for (long long i = 0; i < count; ++i) out[i] = float_to_half(x[i]);
}
void orc_half_to_float(const uint16_t* h, float* out, long long count) {
    for (long long i = 0; i < count; ++i) out[i] = half_to_float(h[i]);
}

/* r = f - A u (float) from binary16 u, f; k32 the float coefficient or NULL */
void orc_residual_f16(int dim, int n, const float* k32, const uint16_t* u, const uint16_t* f, float* r) {
    const Grid<Half> g = make_grid<Half>(dim, n, k32, 1.0);
    residual(g, (const Half*)u, (const Half*)f, r);
}
/* one smoothing sweep in place on binary16 u (smoother as orc_smooth_f64) */
void orc_smooth_f16(int dim, int n, const float* k32, int smoother, double omega, uint16_t* u, const uint16_t* f) {
    const Grid<Half> g = make_grid<Half>(dim, n, k32, omega);
    std::vector<Half> tmp;
    if (smoother == SMOOTH_JACOBI) jacobi_sweep(g, (Half*)u, (const Half*)f, tmp);
    else rbgs_sweep(g, (Half*)u, (const Half*)f, smoother == SMOOTH_RBGS_SYM ? 1 : 0);
}
/* full weighting of a float residual into binary16 coarse cells */
void orc_restrict_f16(int dim, int nf, const float* r, uint16_t* fc) { restrict_fw(dim, nf, r, (Half*)fc); }
void orc_prolong_correct_f16(int dim, int nf, uint16_t* u, const uint16_t* ec) {
    prolong_correct(dim, nf, (Half*)u, (const Half*)ec);
}
int orc_cycle_f16(int dim, int n, const float* k32, int smoother, double omega, int nu1, int nu2, int cycle,
                  int coarse_n, int cg_iters, uint16_t* u, const uint16_t* f) {
    if ((dim != 2 && dim != 3) || !valid_edge(n) || !valid_opts(n, cycle, coarse_n)) return -1;
    Hierarchy<Half> H;
    std::vector<double> k64;
    if (k32) k64.assign(k32, k32 + npts(dim, n));
    build(H, dim, n, k32 ? k64.data() : nullptr, smoother, omega, nu1, nu2, coarse_n);
    H.cycle = cycle;
    H.cg_iters = cg_iters;
    vcycle(H, 0, (Half*)u, (const Half*)f);
    return 0;
}

/* Scale of a residual whose largest magnitude is mx: the power of two s with
 * 8 <= s mx < 16, so that the scaled residual and the correction it induces
 * stay far inside binary16's range (largest finite value 65504, smallest
 * normal 2^-14) whatever the size of the residual; the exponent is kept in
 * [-126, 127] so that s is a normal float (the relation holds for
 * 2^-123 <= mx < 2^130); 1 for a zero or non-finite mx. */
double orc_fp16_scale(double mx) {
    if (!(mx > 0.0) || !std::isfinite(mx)) return 1.0;
    int e;
    (void)std::frexp(mx, &e); /* mx = m 2^e, 1/2 <= m < 1 */
    return std::ldexp(1.0, std::min(127, std::max(-126, 4 - e)));
}

/* One FP64 refinement pass of the half-precision form: when e16 is given,
 * u += e16 / s_prev on inner nodes (e16 holds the correction scaled by
 * s_prev); r = f - A u in FP64; r16 = half(float(s_next) * float(r)) (the
 * residual rounded to float as in the single-precision form, then scaled by
 * a power of two and stored in binary16); *mx = max |r|; returns ||r||_2. */
double orc_ir_update_f16(int dim, int n, const double* k64, double* u, const uint16_t* e16, double s_prev,
                         const double* f, double s_next, uint16_t* r16, double* mx) {
    const Grid<double> g = make_grid<double>(dim, n, k64, 1.0);
    const size_t total = npts(dim, n);
    const int k0 = dim == 3 ? 1 : 0, k1 = dim == 3 ? n - 1 : 1;
    if (e16) {
        const double inv = 1.0 / s_prev;
        for (int k = k0; k < k1; ++k)
            for (int j = 1; j < n - 1; ++j)
                for (int i = 1; i < n - 1; ++i) {
                    const idx_t p = at(dim, n, i, j, k);
                    u[p] = u[p] + (double)half_to_float(e16[p]) * inv;
                }
    }
    std::vector<double> r(total);
    residual(g, u, f, r.data());
    const float s32 = (float)s_next;
    double m = 0.0;
    for (size_t p = 0; p < total; ++p) {
        r16[p] = float_to_half(s32 * (float)r[p]);
        m = std::max(m, std::fabs(r[p]));
    }
    *mx = m;
    return residual_norm(g, u, f);
}

/* Half-precision cycles inside FP64 iterative refinement.  The right-hand
 * side of every cycle is the FP64 residual scaled by orc_fp16_scale of the
 * largest residual magnitude of the previous pass (of the same pass for the
 * first cycle, which is measured once beforehand); the correction is
 * unscaled when it is added.  hist as in orc_solve_ir_mg_f32. */
int orc_solve_ir_mg_f16(int dim, int n, const double* k64, int smoother, double omega, int nu1, int nu2, int cycle,
                        int coarse_n, int cg_iters, double* u, const double* f, double tol, int max_cycles,
                        double* hist, int* cycles) {
    if ((dim != 2 && dim != 3) || !valid_edge(n) || max_cycles < 0 || !valid_opts(n, cycle, coarse_n)) return -1;
    Hierarchy<Half> H;
    build(H, dim, n, k64, smoother, omega, nu1, nu2, coarse_n);
    H.cycle = cycle;
    H.cg_iters = cg_iters;
    const size_t total = npts(dim, n);
    std::vector<Half> e(total, Half(0.0f)), r16(total, Half(0.0f));
    double mx = 0.0;
    (void)orc_ir_update_f16(dim, n, k64, u, nullptr, 1.0, f, 1.0, (uint16_t*)r16.data(), &mx);
    double s = orc_fp16_scale(mx);
    const double rho0 = orc_ir_update_f16(dim, n, k64, u, nullptr, 1.0, f, s, (uint16_t*)r16.data(), &mx);
    if (hist) hist[0] = rho0;
    int it = 0;
    int status = rho0 == 0.0 ? 0 : 1;
    while (status == 1 && it < max_cycles) {
        std::fill(e.begin(), e.end(), Half(0.0f));
        vcycle(H, 0, e.data(), r16.data());
        ++it;
        const double s_next = orc_fp16_scale(mx);
        const double rho = orc_ir_update_f16(dim, n, k64, u, (const uint16_t*)e.data(), s, f, s_next,
                                             (uint16_t*)r16.data(), &mx);
        s = s_next;
        if (hist) hist[it] = rho;
        if (rho <= tol * rho0) status = 0;
        else if (!(rho == rho) || rho > 1e6 * rho0) status = -5;
    }
    if (cycles) *cycles = it;
    return status;
}

/* ------------------------------------------------------------------ */
/* Cell-centred Neumann problems (FP64).  Arrays hold n^dim cell values. */
/* ------------------------------------------------------------------ */

void orc_cc_residual(int dim, int n, const double* u, const double* f, double* r) {
    cc_residual(cc_level(dim, n, 1.0), u, f, r);
}
/* one smoothing sweep in place (0 RBGS red first, 1 Jacobi) */
void orc_cc_smooth(int dim, int n, int smoother, double omega, double* u, const double* f) {
    const CCLevel L = cc_level(dim, n, omega);
    std::vector<double> tmp;
    if (smoother == SMOOTH_JACOBI) cc_jacobi(L, u, f, tmp);
    else cc_rbgs(L, u, f);
}
void orc_cc_restrict(int dim, int nf, const double* r, double* fc) { cc_restrict(dim, nf, r, fc); }
void orc_cc_prolong_correct(int dim, int nf, double* u, const double* ec) { cc_prolong_correct(dim, nf, u, ec); }
double orc_cc_sum(int dim, int n, const double* u) { return cc_sum(dim, n, u); }
double orc_cc_residual_norm(int dim, int n, const double* u, const double* f) {
    return cc_residual_norm(cc_level(dim, n, 1.0), u, f);
}
/* one cycle on u (no mean handling) */
int orc_cc_cycle(int dim, int n, int smoother, double omega, int nu1, int nu2, int cycle, double* u,
                 const double* f) {
    if (!cc_valid(dim, n) || cycle < CYCLE_V || cycle > CYCLE_F) return -1;
    CCHierarchy H;
    cc_build(H, dim, n, smoother, omega, nu1, nu2, cycle);
    cc_cycle(H, 0, u, f, cycle);
    return 0;
}
/* Solve: fh = f - mean(f) (the compatible right-hand side), u -= mean(u);
 * rho_0 = ||fh - A u||; then cycles, each followed by u -= mean(u), until
 * rho_k <= tol rho_0 or max_cycles.  fh_out (may be NULL) receives fh. */
int orc_cc_solve(int dim, int n, int smoother, double omega, int nu1, int nu2, int cycle, double* u,
                 const double* f, double tol, int max_cycles, double* hist, int* cycles, double* fh_out) {
    if (!cc_valid(dim, n) || cycle < CYCLE_V || cycle > CYCLE_F || max_cycles < 0) return -1;
    CCHierarchy H;
    cc_build(H, dim, n, smoother, omega, nu1, nu2, cycle);
    const size_t N = cc_cells(dim, n);
    std::vector<double> fh(f, f + N);
    cc_remove_mean(dim, n, fh.data());
    if (fh_out) std::memcpy(fh_out, fh.data(), N * sizeof(double));
    cc_remove_mean(dim, n, u);
    const CCLevel L0 = cc_level(dim, n, omega);
    const double rho0 = cc_residual_norm(L0, u, fh.data());
    if (hist) hist[0] = rho0;
    int it = 0, status = rho0 == 0.0 ? 0 : 1;
    while (status == 1 && it < max_cycles) {
        cc_cycle(H, 0, u, fh.data(), cycle);
        cc_remove_mean(dim, n, u);
        ++it;
        const double rho = cc_residual_norm(L0, u, fh.data());
        if (hist) hist[it] = rho;
        if (rho <= tol * rho0) status = 0;
        else if (!(rho == rho) || rho > 1e6 * rho0) status = -5;
    }
    if (cycles) *cycles = it;
    return status;
}

/* ------------------------------------------------------------------ */
/* Complex diffusion (FP64).  Complex arrays hold n^dim (re, im) pairs.    */
/* ct, st: cos(theta), sin(theta) as the caller evaluated them.          */
/* ------------------------------------------------------------------ */

/* N(u) with g of u */
void orc_cd_apply(int dim, int n, double tau, double theta, double k, double ct, double st, const double* u,
                  double* out) {
    const CDParams P = cd_params(dim, tau, theta, k, ct, st);
    std::vector<Cx> g;
    const size_t N = cc_cells(dim, n);
    std::vector<Cx> zero(N, Cx{0.0, 0.0});
    std::vector<Cx> r(N);
    cd_residual(P, n, cd_c(n), (const Cx*)u, zero.data(), g, r.data());
    for (size_t p = 0; p < N; ++p) ((Cx*)out)[p] = Cx{-r[p].re, -r[p].im};
}
void orc_cd_g(int dim, int n, double theta, double k, double ct, double st, const double* u, double* g) {
    const CDParams P = cd_params(dim, 1.0, theta, k, ct, st);
    cd_compute_g(P, n, (const Cx*)u, (Cx*)g);
}
void orc_cd_sweep(int dim, int n, double tau, double theta, double k, double ct, double st, int smoother,
                  double omega, double* u, const double* f) {
    const CDParams P = cd_params(dim, tau, theta, k, ct, st);
    std::vector<Cx> g, tmp;
    cd_sweep(P, n, cd_c(n), smoother, omega, (Cx*)u, (const Cx*)f, g, tmp);
}
double orc_cd_residual_norm(int dim, int n, double tau, double theta, double k, double ct, double st,
                            const double* u, const double* f) {
    const CDParams P = cd_params(dim, tau, theta, k, ct, st);
    std::vector<Cx> g, r(cc_cells(dim, n));
    cd_residual(P, n, cd_c(n), (const Cx*)u, (const Cx*)f, g, r.data());
    return cd_norm(dim, n, r.data());
}
/* one FAS cycle on u for N(u) = f */
int orc_cd_fas(int dim, int n, double tau, double theta, double k, double ct, double st, int smoother, double omega,
               int nu1, int nu2, double* u, const double* f) {
    if (!cc_valid(dim, n) || !(tau > 0.0)) return -1;
    CDHierarchy H;
    cd_build(H, cd_params(dim, tau, theta, k, ct, st), n, smoother, omega, nu1, nu2);
    cd_fas(H, 0, (Cx*)u, (const Cx*)f);
    return 0;
}
/* Implicit Euler: 'steps' time steps from u (in: u^0, out: u^steps); step m
 * solves N(u) = u^m / tau by FAS cycles from u^m until ||f - N(u)|| <= tol
 * ||f - N(u^m)|| or max_cycles.  cycles[m] (may be NULL) receives the cycle
 * count of step m, hist (may be NULL, steps * (max_cycles + 1)) the residual
 * norms of each step.  Returns 0, or 1 if some step missed the tolerance. */
int orc_cd_run(int dim, int n, double tau, double theta, double k, double ct, double st, int smoother, double omega,
               int nu1, int nu2, double* u, int steps, double tol, int max_cycles, int* cycles, double* hist) {
    if (!cc_valid(dim, n) || !(tau > 0.0) || steps < 0 || max_cycles < 0) return -1;
    const CDParams P = cd_params(dim, tau, theta, k, ct, st);
    CDHierarchy H;
    cd_build(H, P, n, smoother, omega, nu1, nu2);
    const size_t N = cc_cells(dim, n);
    Cx* U = (Cx*)u;
    std::vector<Cx> f(N), r(N);
    const double c = cd_c(n);
    int status = 0;
    for (int m = 0; m < steps; ++m) {
        for (size_t p = 0; p < N; ++p) f[p] = cx_scale(P.itau, U[p]);
        cd_residual(P, n, c, U, f.data(), H.g, r.data());
        const double rho0 = cd_norm(dim, n, r.data());
        double* hm = hist ? hist + (size_t)m * (size_t)(max_cycles + 1) : nullptr;
        if (hm) hm[0] = rho0;
        int it = 0;
        bool done = rho0 == 0.0;
        while (!done && it < max_cycles) {
            cd_fas(H, 0, U, f.data());
            ++it;
            cd_residual(P, n, c, U, f.data(), H.g, r.data());
            const double rho = cd_norm(dim, n, r.data());
            if (hm) hm[it] = rho;
            done = rho <= tol * rho0;
        }
        if (!done) status = 1;
        if (cycles) cycles[m] = it;
    }
    return status;
}

} /* extern "C" */
