// Constant-stencil operator on node-based Dirichlet grids (Section 2.2: the
// discretisation is a stencil with constant entries; the Laplacian's 5-/7-
// point stencil is one instance):
//   (A u)_p = c (s0 u_p + t),  t = ((sW uW + sE uE) + (sS uS + sN uN)) [+ (sB uB + sT uT)],
// c = 1/h^2 of the level (the same stencil re-discretised on every level),
// relaxation u + wd r with wd = omega h^2 / s0, full-weighting restriction of
// the residual and bi-/trilinear interpolation in the expression order of
// the Laplacian path, the exact solve of the single unknown of the 3-node
// grid.  FP64, plain one-node-per-thread kernels (neighbours through the
// caches): a second operator beside the tuned Laplacian path, not its
// throughput form.
#include <algorithm>
#include <cstring>

#include "mg_kern.h"
#include "mg_st.h"

namespace mg {
namespace {

template <int DIM>
__device__ __forceinline__ void st_ijk(size_t p, int n, int& i, int& j, int& k) {
    i = (int)(p % (size_t)n);
    const size_t q = p / (size_t)n;
    j = (int)(q % (size_t)n);
    k = DIM == 2 ? 0 : (int)(q / (size_t)n);
}

template <int DIM>
__device__ __forceinline__ bool st_inner(int n, int i, int j, int k) {
    return i >= 1 && i <= n - 2 && j >= 1 && j <= n - 2 && (DIM == 2 || (k >= 1 && k <= n - 2));
}

// r_p = f_p - c (s0 u_p + t)
template <int DIM>
__device__ __forceinline__ double st_res(const MG_GLOBAL double* u, const MG_GLOBAL double* f, const STConst& L,
                                         size_t p) {
    const size_t sy = (size_t)L.n, sz = (size_t)L.n * L.n;
    double t = (L.s[1] * u[p - 1] + L.s[2] * u[p + 1]) + (L.s[3] * u[p - sy] + L.s[4] * u[p + sy]);
    if constexpr (DIM == 3) t = t + (L.s[5] * u[p - sz] + L.s[6] * u[p + sz]);
    return f[p] - L.c * (L.s[0] * u[p] + t);
}

template <int DIM, bool JAC>
__global__ __launch_bounds__(NT) void k_st_relax(const double* uin_, double* uout_, const double* __restrict__ f_,
                                                 STConst L, int colour) {
    const MG_GLOBAL double* uin = gp(uin_);
    MG_GLOBAL double* uout = gp(uout_);
    const MG_GLOBAL double* __restrict__ f = gp(f_);
    const int n = L.n;
    const size_t N = DIM == 2 ? (size_t)n * n : (size_t)n * n * n;
    const size_t p = (size_t)blockIdx.x * NT + threadIdx.x;
    if (p >= N) return;
    int i, j, k;
    st_ijk<DIM>(p, n, i, j, k);
    if (!st_inner<DIM>(n, i, j, k)) return;
    if (!JAC && ((i + j + k) & 1) != colour) return;
    const double r = st_res<DIM>(uin, f, L, p);
    uout[p] = uin[p] + L.wd * r;
}

// Full weighting of the residual at each inner coarse node (the residual of
// each of the 3^d fine nodes evaluated where it is needed), in the expression
// order of the Laplacian path's restriction.
template <int DIM>
__global__ __launch_bounds__(NT) void k_st_restrict(const double* __restrict__ u_, const double* __restrict__ f_,
                                                    double* __restrict__ fc_, STConst L) {
    const MG_GLOBAL double* __restrict__ u = gp(u_);
    const MG_GLOBAL double* __restrict__ f = gp(f_);
    const int nf = L.n, nc = (nf - 1) / 2 + 1;
    const size_t Nc = DIM == 2 ? (size_t)nc * nc : (size_t)nc * nc * nc;
    const size_t q = (size_t)blockIdx.x * NT + threadIdx.x;
    if (q >= Nc) return;
    int I, J, K;
    st_ijk<DIM>(q, nc, I, J, K);
    if (!st_inner<DIM>(nc, I, J, K)) return;
    const size_t sx = 1, sy = (size_t)nf, sz = (size_t)nf * nf;
    auto r = [&](size_t p) { return st_res<DIM>(u, f, L, p); };
    double v;
    if constexpr (DIM == 2) {
        const size_t p = (size_t)(2 * J) * nf + (size_t)(2 * I);
        const double edges = (r(p - sx) + r(p + sx)) + (r(p - sy) + r(p + sy));
        const double corners = (r(p - sx - sy) + r(p + sx - sy)) + (r(p - sx + sy) + r(p + sx + sy));
        v = (0.25 * r(p) + 0.125 * edges) + 0.0625 * corners;
    } else {
        const size_t p = ((size_t)(2 * K) * nf + (size_t)(2 * J)) * nf + (size_t)(2 * I);
        const double faces = ((r(p - sx) + r(p + sx)) + (r(p - sy) + r(p + sy))) + (r(p - sz) + r(p + sz));
        const double exy = (r(p - sx - sy) + r(p + sx - sy)) + (r(p - sx + sy) + r(p + sx + sy));
        const double exz = (r(p - sx - sz) + r(p + sx - sz)) + (r(p - sx + sz) + r(p + sx + sz));
        const double eyz = (r(p - sy - sz) + r(p + sy - sz)) + (r(p - sy + sz) + r(p + sy + sz));
        const double edges = (exy + exz) + eyz;
        const double cz0 = (r(p - sx - sy - sz) + r(p + sx - sy - sz)) + (r(p - sx + sy - sz) + r(p + sx + sy - sz));
        const double cz1 = (r(p - sx - sy + sz) + r(p + sx - sy + sz)) + (r(p - sx + sy + sz) + r(p + sx + sy + sz));
        const double corners = cz0 + cz1;
        v = ((0.125 * r(p) + 0.0625 * faces) + 0.03125 * edges) + 0.015625 * corners;
    }
    gp(fc_)[q] = v;
}

// u += P ec at inner fine nodes: coincident value, or the mean of 2 / 4 / 8
// coarse neighbours along the odd axes (taken in x, y, z order)
template <int DIM>
__global__ __launch_bounds__(NT) void k_st_prolong(double* __restrict__ u_, const double* __restrict__ ec_, int nf) {
    MG_GLOBAL double* __restrict__ u = gp(u_);
    const MG_GLOBAL double* __restrict__ e = gp(ec_);
    const size_t N = DIM == 2 ? (size_t)nf * nf : (size_t)nf * nf * nf;
    const size_t p = (size_t)blockIdx.x * NT + threadIdx.x;
    if (p >= N) return;
    int i, j, k;
    st_ijk<DIM>(p, nf, i, j, k);
    if (!st_inner<DIM>(nf, i, j, k)) return;
    const int nc = (nf - 1) / 2 + 1;
    const size_t q = ((size_t)(k / 2) * nc + (size_t)(j / 2)) * nc + (size_t)(i / 2);
    size_t s[3];
    int m = 0;
    if (i & 1) s[m++] = 1;
    if (j & 1) s[m++] = (size_t)nc;
    if (DIM == 3 && (k & 1)) s[m++] = (size_t)nc * nc;
    double v;
    if (m == 0) v = e[q];
    else if (m == 1) v = 0.5 * (e[q] + e[q + s[0]]);
    else if (m == 2) v = 0.25 * ((e[q] + e[q + s[0]]) + (e[q + s[1]] + e[q + s[0] + s[1]]));
    else
        v = 0.125 * (((e[q] + e[q + s[0]]) + (e[q + s[1]] + e[q + s[0] + s[1]])) +
                     ((e[q + s[2]] + e[q + s[0] + s[2]]) + (e[q + s[1] + s[2]] + e[q + s[0] + s[1] + s[2]])));
    u[p] = u[p] + v;
}

template <int DIM>
__global__ void k_st_coarsest(double* __restrict__ u_, const double* __restrict__ f_, STConst L) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const size_t p = DIM == 2 ? 4 : 13;  // centre of the 3-node grid
    gp(u_)[p] = gp(f_)[p] / (L.c * L.s[0]);
}

// per-block partial sums of r^2 over inner nodes
template <int DIM>
__global__ __launch_bounds__(NT) void k_st_norm(const double* __restrict__ u_, const double* __restrict__ f_,
                                                STConst L, double* __restrict__ part) {
    __shared__ double red4[4];
    const int n = L.n;
    const size_t N = DIM == 2 ? (size_t)n * n : (size_t)n * n * n;
    const size_t p = (size_t)blockIdx.x * NT + threadIdx.x;
    double acc = 0.0;
    if (p < N) {
        int i, j, k;
        st_ijk<DIM>(p, n, i, j, k);
        if (st_inner<DIM>(n, i, j, k)) {
            const double r = st_res<DIM>(gp(u_), gp(f_), L, p);
            acc = r * r;
        }
    }
    const double s = block_sum(acc, red4);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

inline unsigned nblk(size_t N) { return (unsigned)((N + NT - 1) / NT); }
inline size_t nodes(int dim, int n) { return dim == 2 ? (size_t)n * n : (size_t)n * n * n; }

}  // namespace

STConst st_const(int dim, int n, const double* stencil, double omega) {
    STConst L;
    std::memset(&L, 0, sizeof(L));
    L.n = n;
    const double h = 1.0 / (double)(n - 1);
    L.c = 1.0 / (h * h);
    L.wd = (omega * (h * h)) / stencil[0];
    for (int q = 0; q < 2 * dim + 1; ++q) L.s[q] = stencil[q];
    return L;
}

hipError_t st_relax(int dim, bool jacobi, const double* uin, double* uout, const double* f, const STConst& L,
                    int colour, hipStream_t s) {
    const unsigned b = nblk(nodes(dim, L.n));
    if (dim == 2) {
        if (jacobi) k_st_relax<2, true><<<b, NT, 0, s>>>(uin, uout, f, L, colour);
        else k_st_relax<2, false><<<b, NT, 0, s>>>(uin, uout, f, L, colour);
    } else {
        if (jacobi) k_st_relax<3, true><<<b, NT, 0, s>>>(uin, uout, f, L, colour);
        else k_st_relax<3, false><<<b, NT, 0, s>>>(uin, uout, f, L, colour);
    }
    return hipGetLastError();
}

hipError_t st_restrict(int dim, const double* u, const double* f, double* fc, const STConst& L, hipStream_t s) {
    const unsigned b = nblk(nodes(dim, (L.n - 1) / 2 + 1));
    if (dim == 2) k_st_restrict<2><<<b, NT, 0, s>>>(u, f, fc, L);
    else k_st_restrict<3><<<b, NT, 0, s>>>(u, f, fc, L);
    return hipGetLastError();
}

hipError_t st_prolong(int dim, double* u, const double* ec, int n, hipStream_t s) {
    const unsigned b = nblk(nodes(dim, n));
    if (dim == 2) k_st_prolong<2><<<b, NT, 0, s>>>(u, ec, n);
    else k_st_prolong<3><<<b, NT, 0, s>>>(u, ec, n);
    return hipGetLastError();
}

hipError_t st_coarsest(int dim, double* u, const double* f, const STConst& L, hipStream_t s) {
    if (dim == 2) k_st_coarsest<2><<<1, 64, 0, s>>>(u, f, L);
    else k_st_coarsest<3><<<1, 64, 0, s>>>(u, f, L);
    return hipGetLastError();
}

int st_norm_parts(int dim, int n) { return (int)nblk(nodes(dim, n)); }

hipError_t st_norm(int dim, const double* u, const double* f, const STConst& L, double* part, double* norm,
                   hipStream_t s) {
    const int np = st_norm_parts(dim, L.n);
    if (dim == 2) k_st_norm<2><<<np, NT, 0, s>>>(u, f, L, part);
    else k_st_norm<3><<<np, NT, 0, s>>>(u, f, L, part);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_norm_finalize(part, np, np, 0, 1, norm, s);
}

}  // namespace mg
