// Cell-centred grids with a homogeneous Neumann boundary (Table 1: cell-
// centred discretisation, Neumann boundary condition, constant interpolation;
// the boundary of the complex-diffusion application of Section 4).
//
// n = 2^L cells per axis, h = 1/n, one FP64 value per cell (no ghost cells),
// x fastest.  Zero flux through the boundary: a neighbour outside the domain
// takes the cell's own value, so
//   (A u)_p = c (2d u_p - s),  s = ((uW+uE)+(uS+uN))[+(uB+uT)] with ghosts,
// relaxation u + wd[m] r with wd[m] = omega h^2 / (2d - m) (m = faces of the
// cell on the boundary: omega over the true diagonal), restriction by the
// average of the 2^d children, constant interpolation, a single-cell
// coarsest level (zero correction).  The operator is singular: the solve
// projects f onto mean zero and keeps the iterate at mean zero, with sums in
// a fixed order (each x-row left to right, the rows of a plane, the planes).
//
// These are plain one-cell-per-thread kernels (neighbours through the
// caches): the cell-centred path is a second discretisation beside the
// node-based hot path, not its throughput form.
#include <algorithm>
#include <cstring>

#include "mg_cc.h"
#include "mg_kern.h"

namespace mg {
namespace {

template <int DIM>
__device__ __forceinline__ double cc_apply(const MG_GLOBAL double* u, int n, double c, int i, int j, int k,
                                           size_t p) {
    const double uC = u[p];
    const double uW = i > 0 ? u[p - 1] : uC, uE = i < n - 1 ? u[p + 1] : uC;
    const double uS = j > 0 ? u[p - n] : uC, uN = j < n - 1 ? u[p + n] : uC;
    if constexpr (DIM == 2) {
        return c * (4.0 * uC - ((uW + uE) + (uS + uN)));
    } else {
        const size_t sz = (size_t)n * n;
        const double uB = k > 0 ? u[p - sz] : uC, uT = k < n - 1 ? u[p + sz] : uC;
        return c * (6.0 * uC - (((uW + uE) + (uS + uN)) + (uB + uT)));
    }
}

template <int DIM>
__device__ __forceinline__ void cc_ijk(size_t p, int n, int& i, int& j, int& k) {
    i = (int)(p % (size_t)n);
    const size_t q = p / (size_t)n;
    j = (int)(q % (size_t)n);
    k = DIM == 2 ? 0 : (int)(q / (size_t)n);
}

// RBGS colour (in place; a colour reads only the other colour) or Jacobi
// (out of place) relaxation of every cell of one level.
template <int DIM, bool JAC>
__global__ __launch_bounds__(NT) void k_cc_relax(const double* uin_, double* uout_,
                                                 const double* __restrict__ f_, CCConst L, int colour) {
    const MG_GLOBAL double* uin = gp(uin_);
    MG_GLOBAL double* uout = gp(uout_);
    const MG_GLOBAL double* __restrict__ f = gp(f_);
    const int n = L.n;
    const size_t N = DIM == 2 ? (size_t)n * n : (size_t)n * n * n;
    const size_t p = (size_t)blockIdx.x * NT + threadIdx.x;
    if (p >= N) return;
    int i, j, k;
    cc_ijk<DIM>(p, n, i, j, k);
    if (!JAC && ((i + j + k) & 1) != colour) return;
    int m = (i == 0) + (i == n - 1) + (j == 0) + (j == n - 1);
    if (DIM == 3) m += (k == 0) + (k == n - 1);
    const double r = f[p] - cc_apply<DIM>(uin, n, L.c, i, j, k, p);
    uout[p] = uin[p] + L.wd[m] * r;
}

// fc = average of the residuals of the 2^d children of each coarse cell
template <int DIM>
__global__ __launch_bounds__(NT) void k_cc_restrict(const double* __restrict__ u_, const double* __restrict__ f_,
                                                    double* __restrict__ fc_, CCConst L) {
    const MG_GLOBAL double* __restrict__ u = gp(u_);
    const MG_GLOBAL double* __restrict__ f = gp(f_);
    const int n = L.n, nc = n / 2;
    const size_t Nc = DIM == 2 ? (size_t)nc * nc : (size_t)nc * nc * nc;
    const size_t q = (size_t)blockIdx.x * NT + threadIdx.x;
    if (q >= Nc) return;
    int I, J, K;
    cc_ijk<DIM>(q, nc, I, J, K);
    auto res = [&](int i, int j, int k) {
        const size_t p = ((size_t)k * n + j) * n + i;
        return f[p] - cc_apply<DIM>(u, n, L.c, i, j, k, p);
    };
    const int i = 2 * I, j = 2 * J, k = 2 * K;
    const double q0 = (res(i, j, k) + res(i + 1, j, k)) + (res(i, j + 1, k) + res(i + 1, j + 1, k));
    double v;
    if constexpr (DIM == 2) {
        v = 0.25 * q0;
    } else {
        const double q1 = (res(i, j, k + 1) + res(i + 1, j, k + 1)) + (res(i, j + 1, k + 1) + res(i + 1, j + 1, k + 1));
        v = 0.125 * (q0 + q1);
    }
    gp(fc_)[q] = v;
}

// u += e(parent) (constant interpolation)
template <int DIM>
__global__ __launch_bounds__(NT) void k_cc_prolong(double* __restrict__ u_, const double* __restrict__ ec_, int n) {
    const size_t N = DIM == 2 ? (size_t)n * n : (size_t)n * n * n;
    const size_t p = (size_t)blockIdx.x * NT + threadIdx.x;
    if (p >= N) return;
    int i, j, k;
    cc_ijk<DIM>(p, n, i, j, k);
    const int nc = n / 2;
    const size_t q = ((size_t)(k / 2) * nc + j / 2) * nc + i / 2;
    MG_GLOBAL double* u = gp(u_);
    u[p] = u[p] + gp(ec_)[q];
}

__global__ __launch_bounds__(NT) void k_cc_fill(double* __restrict__ v, size_t N, double x) {
    const size_t p = (size_t)blockIdx.x * NT + threadIdx.x;
    if (p < N) gp(v)[p] = x;
}

// Sums in the fixed order: rows[t] = sum over x of row t (left to right).
__global__ __launch_bounds__(NT) void k_cc_rows(const double* __restrict__ v_, int n, size_t nrows,
                                                double* __restrict__ rows) {
    const size_t t = (size_t)blockIdx.x * NT + threadIdx.x;
    if (t >= nrows) return;
    const MG_GLOBAL double* __restrict__ v = gp(v_) + t * (size_t)n;
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += v[i];
    gp(rows)[t] = s;
}
// planes[k] = sum of the n row sums of plane k in order (3D)
__global__ __launch_bounds__(NT) void k_cc_planes(const double* __restrict__ rows_, int n, double* __restrict__ planes) {
    const int k = blockIdx.x * NT + threadIdx.x;
    if (k >= n) return;
    const MG_GLOBAL double* __restrict__ rows = gp(rows_) + (size_t)k * n;
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += rows[j];
    gp(planes)[k] = s;
}
// out[0] = (sum of parts[0..cnt) in order) / N
__global__ void k_cc_mean(const double* __restrict__ parts, int cnt, double N, double* __restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int t = 0; t < cnt; ++t) s += parts[t];
    out[0] = s / N;
}
__global__ __launch_bounds__(NT) void k_cc_sub(double* __restrict__ v_, size_t N, const double* __restrict__ mean) {
    const size_t p = (size_t)blockIdx.x * NT + threadIdx.x;
    if (p >= N) return;
    MG_GLOBAL double* v = gp(v_);
    v[p] = v[p] - *gp(mean);
}

// per-block partial sums of r^2 (the residual norm; any summation order)
template <int DIM>
__global__ __launch_bounds__(NT) void k_cc_norm(const double* __restrict__ u_, const double* __restrict__ f_,
                                                CCConst L, double* __restrict__ part) {
    __shared__ double red4[4];
    const MG_GLOBAL double* __restrict__ u = gp(u_);
    const int n = L.n;
    const size_t N = DIM == 2 ? (size_t)n * n : (size_t)n * n * n;
    const size_t p = (size_t)blockIdx.x * NT + threadIdx.x;
    double acc = 0.0;
    if (p < N) {
        int i, j, k;
        cc_ijk<DIM>(p, n, i, j, k);
        const double r = gp(f_)[p] - cc_apply<DIM>(u, n, L.c, i, j, k, p);
        acc = r * r;
    }
    const double s = block_sum(acc, red4);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

inline unsigned blocks_for(size_t N) { return (unsigned)((N + NT - 1) / NT); }

}  // namespace

size_t cc_cells(int dim, int n) { return dim == 2 ? (size_t)n * n : (size_t)n * n * n; }

CCConst cc_const(int dim, int n, double omega) {
    CCConst L;
    L.n = n;
    const double h = 1.0 / (double)n;
    L.c = 1.0 / (h * h);
    for (int m = 0; m < 4; ++m) L.wd[m] = (omega * (h * h)) / (double)(2 * dim - m);
    return L;
}

hipError_t cc_relax(int dim, bool jacobi, const double* uin, double* uout, const double* f, CCConst L, int colour,
                    hipStream_t s) {
    const unsigned b = blocks_for(cc_cells(dim, L.n));
    if (dim == 2) {
        if (jacobi) k_cc_relax<2, true><<<b, NT, 0, s>>>(uin, uout, f, L, colour);
        else k_cc_relax<2, false><<<b, NT, 0, s>>>(uin, uout, f, L, colour);
    } else {
        if (jacobi) k_cc_relax<3, true><<<b, NT, 0, s>>>(uin, uout, f, L, colour);
        else k_cc_relax<3, false><<<b, NT, 0, s>>>(uin, uout, f, L, colour);
    }
    return hipGetLastError();
}

hipError_t cc_restrict(int dim, const double* u, const double* f, double* fc, CCConst L, hipStream_t s) {
    const unsigned b = blocks_for(cc_cells(dim, L.n / 2));
    if (dim == 2) k_cc_restrict<2><<<b, NT, 0, s>>>(u, f, fc, L);
    else k_cc_restrict<3><<<b, NT, 0, s>>>(u, f, fc, L);
    return hipGetLastError();
}

hipError_t cc_prolong(int dim, double* u, const double* ec, int n, hipStream_t s) {
    const unsigned b = blocks_for(cc_cells(dim, n));
    if (dim == 2) k_cc_prolong<2><<<b, NT, 0, s>>>(u, ec, n);
    else k_cc_prolong<3><<<b, NT, 0, s>>>(u, ec, n);
    return hipGetLastError();
}

hipError_t cc_fill(double* v, size_t N, double x, hipStream_t s) {
    if (N) k_cc_fill<<<blocks_for(N), NT, 0, s>>>(v, N, x);
    return hipGetLastError();
}

hipError_t cc_mean(int dim, int n, const double* v, double* work, double* mean, hipStream_t s) {
    const size_t nrows = dim == 2 ? (size_t)n : (size_t)n * n;
    k_cc_rows<<<blocks_for(nrows), NT, 0, s>>>(v, n, nrows, work);
    const double N = (double)cc_cells(dim, n);
    if (dim == 2) {
        k_cc_mean<<<1, 64, 0, s>>>(work, n, N, mean);
    } else {
        k_cc_planes<<<blocks_for((size_t)n), NT, 0, s>>>(work, n, work + nrows);
        k_cc_mean<<<1, 64, 0, s>>>(work + nrows, n, N, mean);
    }
    return hipGetLastError();
}

hipError_t cc_remove_mean(int dim, int n, double* v, double* work, double* mean, hipStream_t s) {
    hipError_t e = cc_mean(dim, n, v, work, mean, s);
    if (e != hipSuccess) return e;
    const size_t N = cc_cells(dim, n);
    k_cc_sub<<<blocks_for(N), NT, 0, s>>>(v, N, mean);
    return hipGetLastError();
}

int cc_norm_parts(int dim, int n) { return (int)blocks_for(cc_cells(dim, n)); }

hipError_t cc_norm(int dim, const double* u, const double* f, CCConst L, double* part, double* norm, hipStream_t s) {
    const int nparts = cc_norm_parts(dim, L.n);
    if (dim == 2) k_cc_norm<2><<<nparts, NT, 0, s>>>(u, f, L, part);
    else k_cc_norm<3><<<nparts, NT, 0, s>>>(u, f, L, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_norm_finalize(part, nparts, nparts, 0, 1, norm, s);
}

size_t cc_work_doubles(int dim, int n) { return (dim == 2 ? (size_t)n : (size_t)n * n) + (size_t)n; }

}  // namespace mg
