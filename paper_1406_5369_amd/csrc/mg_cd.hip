// Complex diffusion (Section 4, Eq. (2)): u_t = div(g(Im u) grad u) with the
// complex diffusivity g(s) = e^{i theta} / (1 + (s / (k theta))^2), a
// homogeneous Neumann boundary, averaged finite differences on a cell-centred
// grid (face diffusivity = mean of the two cells' g), implicit Euler in time
// and, per time step, the full approximation scheme (FAS) with lagged
// diffusivity: every smoothing sweep and every residual uses g of the
// iterate it starts from.  Transfers: averaging restriction (of the residual
// and of the full approximation), constant interpolation of the coarse
// correction.  Complex values are (re, im) pairs of doubles, 16-byte
// aligned, and every complex operation is written out in one fixed order
// (products (ac - bd, ad + bc), quotients ((ac + bd)/|b|^2, (bc - ad)/|b|^2)).
//
// Per time step m: f = u^m / tau and FAS cycles on N(u) = u / tau - div(g grad u)
// = f from u = u^m.  On a level: nu1 sweeps, r = f - N(u), uh = R u, fc =
// N_c(uh) + R r, the coarse cycle from uc = uh, u += P (uc - uh), nu2 sweeps;
// the coarsest level is one cell, N(u) = u / tau, solved exactly.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "mg_cd.h"
#include "mg_kern.h"

namespace mg {
namespace {

struct __attribute__((aligned(16))) Cx {
    double re, im;
};
__device__ __forceinline__ Cx cx_add(Cx a, Cx b) { return Cx{a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ Cx cx_sub(Cx a, Cx b) { return Cx{a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ Cx cx_mul(Cx a, Cx b) { return Cx{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ Cx cx_div(Cx a, Cx b) {
    const double den = b.re * b.re + b.im * b.im;
    return Cx{(a.re * b.re + a.im * b.im) / den, (a.im * b.re - a.re * b.im) / den};
}
__device__ __forceinline__ Cx cx_scale(double s, Cx a) { return Cx{s * a.re, s * a.im}; }

// One 16-byte access per complex value (a struct cannot be copied out of the
// global address space directly).
typedef double d2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ Cx ldc(const MG_GLOBAL Cx* a, size_t p) {
    const d2v v = ((const MG_GLOBAL d2v*)a)[p];
    return Cx{v.x, v.y};
}
__device__ __forceinline__ void stc(MG_GLOBAL Cx* a, size_t p, Cx c) {
    d2v v;
    v.x = c.re;
    v.y = c.im;
    ((MG_GLOBAL d2v*)a)[p] = v;
}

__device__ __forceinline__ Cx cd_g(const CDConst& K, Cx u) {
    const double s = u.im / K.ktheta;
    const double q = 1.0 / (1.0 + s * s);
    return Cx{K.ct * q, K.st * q};
}

template <int DIM>
__device__ __forceinline__ void cd_ijk(size_t p, int n, int& i, int& j, int& k) {
    i = (int)(p % (size_t)n);
    const size_t q = p / (size_t)n;
    j = (int)(q % (size_t)n);
    k = DIM == 2 ? 0 : (int)(q / (size_t)n);
}

// Flux sum F and diagonal sum S of cell p (faces W, E, S, N[, B, T] paired as
// ((W+E)+(S+N))+(B+T); a boundary face contributes zeros).
template <int DIM>
__device__ __forceinline__ void cd_faces(const MG_GLOBAL Cx* u, const MG_GLOBAL Cx* g, int n, int i, int j, int k,
                                         size_t p, Cx& F, Cx& S) {
    const Cx up = ldc(u, p), gq0 = ldc(g, p);
    const Cx zero{0.0, 0.0};
    auto face = [&](bool inside, size_t q, Cx& t, Cx& gf) {
        if (!inside) {
            t = zero;
            gf = zero;
            return;
        }
        const Cx gq = ldc(g, q);
        gf = Cx{0.5 * (gq0.re + gq.re), 0.5 * (gq0.im + gq.im)};
        t = cx_mul(gf, cx_sub(ldc(u, q), up));
    };
    Cx tW, tE, tS, tN, gW, gE, gS, gN;
    face(i > 0, p - 1, tW, gW);
    face(i < n - 1, p + 1, tE, gE);
    face(j > 0, p - (size_t)n, tS, gS);
    face(j < n - 1, p + (size_t)n, tN, gN);
    F = cx_add(cx_add(tW, tE), cx_add(tS, tN));
    S = cx_add(cx_add(gW, gE), cx_add(gS, gN));
    if constexpr (DIM == 3) {
        const size_t sz = (size_t)n * n;
        Cx tB, tT, gB, gT;
        face(k > 0, p - sz, tB, gB);
        face(k < n - 1, p + sz, tT, gT);
        F = cx_add(F, cx_add(tB, tT));
        S = cx_add(S, cx_add(gB, gT));
    }
}

template <int DIM>
__device__ __forceinline__ Cx cd_apply(const MG_GLOBAL Cx* u, const MG_GLOBAL Cx* g, int n, double c, double itau,
                                       int i, int j, int k, size_t p) {
    Cx F, S;
    cd_faces<DIM>(u, g, n, i, j, k, p, F, S);
    const Cx up = ldc(u, p);
    return Cx{itau * up.re - c * F.re, itau * up.im - c * F.im};
}

__global__ __launch_bounds__(NT) void k_cd_g(const Cx* __restrict__ u, Cx* __restrict__ g, size_t N, CDConst K) {
    const size_t p = (size_t)blockIdx.x * NT + threadIdx.x;
    if (p < N) stc(gp(g), p, cd_g(K, ldc(gp(u), p)));
}

// RBGS colour in place (uin == uout) or Jacobi (out of place), g frozen.
template <int DIM, bool JAC>
__global__ __launch_bounds__(NT) void k_cd_relax(const Cx* uin_, Cx* uout_, const Cx* __restrict__ f_,
                                                 const Cx* __restrict__ g_, CDConst K, CDLevel L, int colour) {
    const int n = L.n;
    const size_t N = DIM == 2 ? (size_t)n * n : (size_t)n * n * n;
    const size_t p = (size_t)blockIdx.x * NT + threadIdx.x;
    if (p >= N) return;
    int i, j, k;
    cd_ijk<DIM>(p, n, i, j, k);
    if (!JAC && ((i + j + k) & 1) != colour) return;
    const MG_GLOBAL Cx* uin = gp(uin_);
    Cx F, S;
    cd_faces<DIM>(uin, gp(g_), n, i, j, k, p, F, S);
    const Cx up = ldc(uin, p);
    const Cx Nu{K.itau * up.re - L.c * F.re, K.itau * up.im - L.c * F.im};
    const Cx r = cx_sub(ldc(gp(f_), p), Nu);
    const Cx D{K.itau + L.c * S.re, L.c * S.im};
    stc(gp(uout_), p, cx_add(up, cx_scale(K.omega, cx_div(r, D))));
}

// Per coarse cell: uh = average of the children's u, rc = average of the
// children's residuals f - N(u) (g of u), componentwise in the order of the
// cell-centred restriction.
template <int DIM>
__global__ __launch_bounds__(NT) void k_cd_restrict(const Cx* __restrict__ u_, const Cx* __restrict__ f_,
                                                    const Cx* __restrict__ g_, Cx* __restrict__ uh_,
                                                    Cx* __restrict__ rc_, CDConst K, CDLevel L) {
    const int n = L.n, nc = n / 2;
    const size_t Nc = DIM == 2 ? (size_t)nc * nc : (size_t)nc * nc * nc;
    const size_t q = (size_t)blockIdx.x * NT + threadIdx.x;
    if (q >= Nc) return;
    int I, J, KK;
    cd_ijk<DIM>(q, nc, I, J, KK);
    const MG_GLOBAL Cx* u = gp(u_);
    const MG_GLOBAL Cx* f = gp(f_);
    const MG_GLOBAL Cx* g = gp(g_);
    auto at = [&](int i, int j, int k) { return ((size_t)k * n + j) * n + i; };
    auto res = [&](int i, int j, int k) {
        const size_t p = at(i, j, k);
        return cx_sub(ldc(f, p), cd_apply<DIM>(u, g, n, L.c, K.itau, i, j, k, p));
    };
    const int i = 2 * I, j = 2 * J, k = 2 * KK;
    const Cx r00 = res(i, j, k), r10 = res(i + 1, j, k), r01 = res(i, j + 1, k), r11 = res(i + 1, j + 1, k);
    const Cx u00 = ldc(u, at(i, j, k)), u10 = ldc(u, at(i + 1, j, k)), u01 = ldc(u, at(i, j + 1, k)),
             u11 = ldc(u, at(i + 1, j + 1, k));
    const Cx rq0 = cx_add(cx_add(r00, r10), cx_add(r01, r11));
    const Cx uq0 = cx_add(cx_add(u00, u10), cx_add(u01, u11));
    Cx rv, uv;
    if constexpr (DIM == 2) {
        rv = cx_scale(0.25, rq0);
        uv = cx_scale(0.25, uq0);
    } else {
        const Cx s00 = res(i, j, k + 1), s10 = res(i + 1, j, k + 1), s01 = res(i, j + 1, k + 1),
                 s11 = res(i + 1, j + 1, k + 1);
        const Cx v00 = ldc(u, at(i, j, k + 1)), v10 = ldc(u, at(i + 1, j, k + 1)), v01 = ldc(u, at(i, j + 1, k + 1)),
                 v11 = ldc(u, at(i + 1, j + 1, k + 1));
        const Cx rq1 = cx_add(cx_add(s00, s10), cx_add(s01, s11));
        const Cx uq1 = cx_add(cx_add(v00, v10), cx_add(v01, v11));
        rv = cx_scale(0.125, cx_add(rq0, rq1));
        uv = cx_scale(0.125, cx_add(uq0, uq1));
    }
    stc(gp(rc_), q, rv);
    stc(gp(uh_), q, uv);
}

// fc = N_c(uh) + rc (in place over rc), uc = uh; gc = g(uh)
template <int DIM>
__global__ __launch_bounds__(NT) void k_cd_coarse_rhs(const Cx* __restrict__ uh_, const Cx* __restrict__ gc_,
                                                      Cx* __restrict__ fc_, Cx* __restrict__ uc_, CDConst K,
                                                      CDLevel L) {
    const int n = L.n;
    const size_t N = DIM == 2 ? (size_t)n * n : (size_t)n * n * n;
    const size_t p = (size_t)blockIdx.x * NT + threadIdx.x;
    if (p >= N) return;
    int i, j, k;
    cd_ijk<DIM>(p, n, i, j, k);
    const MG_GLOBAL Cx* uh = gp(uh_);
    const Cx Nv = cd_apply<DIM>(uh, gp(gc_), n, L.c, K.itau, i, j, k, p);
    MG_GLOBAL Cx* fc = gp(fc_);
    stc(fc, p, cx_add(Nv, ldc(fc, p)));
    stc(gp(uc_), p, ldc(uh, p));
}

// u += uc(parent) - uh(parent)
template <int DIM>
__global__ __launch_bounds__(NT) void k_cd_prolong(Cx* __restrict__ u_, const Cx* __restrict__ uc_,
                                                   const Cx* __restrict__ uh_, int n) {
    const size_t N = DIM == 2 ? (size_t)n * n : (size_t)n * n * n;
    const size_t p = (size_t)blockIdx.x * NT + threadIdx.x;
    if (p >= N) return;
    int i, j, k;
    cd_ijk<DIM>(p, n, i, j, k);
    const int nc = n / 2;
    const size_t q = ((size_t)(k / 2) * nc + j / 2) * nc + i / 2;
    MG_GLOBAL Cx* u = gp(u_);
    stc(u, p, cx_add(ldc(u, p), cx_sub(ldc(gp(uc_), q), ldc(gp(uh_), q))));
}

// out = s * a (the coarsest solve u = tau f, the time-step right-hand side f = u / tau)
__global__ __launch_bounds__(NT) void k_cd_scale(const Cx* __restrict__ a, Cx* __restrict__ out, size_t N, double s) {
    const size_t p = (size_t)blockIdx.x * NT + threadIdx.x;
    if (p < N) stc(gp(out), p, cx_scale(s, ldc(gp(a), p)));
}

// out = N(u) (g of u precomputed)
template <int DIM>
__global__ __launch_bounds__(NT) void k_cd_apply(const Cx* __restrict__ u_, const Cx* __restrict__ g_,
                                                 Cx* __restrict__ out, CDConst K, CDLevel L) {
    const int n = L.n;
    const size_t N = DIM == 2 ? (size_t)n * n : (size_t)n * n * n;
    const size_t p = (size_t)blockIdx.x * NT + threadIdx.x;
    if (p >= N) return;
    int i, j, k;
    cd_ijk<DIM>(p, n, i, j, k);
    stc(gp(out), p, cd_apply<DIM>(gp(u_), gp(g_), n, L.c, K.itau, i, j, k, p));
}

// per-block partial sums of |f - N(u)|^2 (re^2 + im^2)
template <int DIM>
__global__ __launch_bounds__(NT) void k_cd_norm(const Cx* __restrict__ u_, const Cx* __restrict__ f_,
                                                const Cx* __restrict__ g_, CDConst K, CDLevel L,
                                                double* __restrict__ part) {
    __shared__ double red4[4];
    const int n = L.n;
    const size_t N = DIM == 2 ? (size_t)n * n : (size_t)n * n * n;
    const size_t p = (size_t)blockIdx.x * NT + threadIdx.x;
    double acc = 0.0;
    if (p < N) {
        int i, j, k;
        cd_ijk<DIM>(p, n, i, j, k);
        const Cx r = cx_sub(ldc(gp(f_), p), cd_apply<DIM>(gp(u_), gp(g_), n, L.c, K.itau, i, j, k, p));
        acc = r.re * r.re + r.im * r.im;
    }
    const double s = block_sum(acc, red4);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

inline unsigned nblk(size_t N) { return (unsigned)((N + NT - 1) / NT); }
inline size_t ncells(int dim, int n) { return dim == 2 ? (size_t)n * n : (size_t)n * n * n; }

}  // namespace

CDLevel cd_level(int n) {
    CDLevel L;
    L.n = n;
    const double h = 1.0 / (double)n;
    L.c = 1.0 / (h * h);
    return L;
}

hipError_t cd_compute_g(const void* u, void* g, size_t N, CDConst K, hipStream_t s) {
    if (N) k_cd_g<<<nblk(N), NT, 0, s>>>((const Cx*)u, (Cx*)g, N, K);
    return hipGetLastError();
}

hipError_t cd_relax(int dim, bool jacobi, const void* uin, void* uout, const void* f, const void* g, CDConst K,
                    CDLevel L, int colour, hipStream_t s) {
    const unsigned b = nblk(ncells(dim, L.n));
    auto ui = (const Cx*)uin;
    auto uo = (Cx*)uout;
    auto ff = (const Cx*)f;
    auto gg = (const Cx*)g;
    if (dim == 2) {
        if (jacobi) k_cd_relax<2, true><<<b, NT, 0, s>>>(ui, uo, ff, gg, K, L, colour);
        else k_cd_relax<2, false><<<b, NT, 0, s>>>(ui, uo, ff, gg, K, L, colour);
    } else {
        if (jacobi) k_cd_relax<3, true><<<b, NT, 0, s>>>(ui, uo, ff, gg, K, L, colour);
        else k_cd_relax<3, false><<<b, NT, 0, s>>>(ui, uo, ff, gg, K, L, colour);
    }
    return hipGetLastError();
}

hipError_t cd_restrict(int dim, const void* u, const void* f, const void* g, void* uh, void* rc, CDConst K,
                       CDLevel L, hipStream_t s) {
    const unsigned b = nblk(ncells(dim, L.n / 2));
    if (dim == 2)
        k_cd_restrict<2><<<b, NT, 0, s>>>((const Cx*)u, (const Cx*)f, (const Cx*)g, (Cx*)uh, (Cx*)rc, K, L);
    else
        k_cd_restrict<3><<<b, NT, 0, s>>>((const Cx*)u, (const Cx*)f, (const Cx*)g, (Cx*)uh, (Cx*)rc, K, L);
    return hipGetLastError();
}

hipError_t cd_coarse_rhs(int dim, const void* uh, const void* gc, void* fc, void* uc, CDConst K, CDLevel Lc,
                         hipStream_t s) {
    const unsigned b = nblk(ncells(dim, Lc.n));
    if (dim == 2)
        k_cd_coarse_rhs<2><<<b, NT, 0, s>>>((const Cx*)uh, (const Cx*)gc, (Cx*)fc, (Cx*)uc, K, Lc);
    else
        k_cd_coarse_rhs<3><<<b, NT, 0, s>>>((const Cx*)uh, (const Cx*)gc, (Cx*)fc, (Cx*)uc, K, Lc);
    return hipGetLastError();
}

hipError_t cd_prolong(int dim, void* u, const void* uc, const void* uh, int n, hipStream_t s) {
    const unsigned b = nblk(ncells(dim, n));
    if (dim == 2) k_cd_prolong<2><<<b, NT, 0, s>>>((Cx*)u, (const Cx*)uc, (const Cx*)uh, n);
    else k_cd_prolong<3><<<b, NT, 0, s>>>((Cx*)u, (const Cx*)uc, (const Cx*)uh, n);
    return hipGetLastError();
}

hipError_t cd_scale(const void* a, void* out, size_t N, double sc, hipStream_t s) {
    if (N) k_cd_scale<<<nblk(N), NT, 0, s>>>((const Cx*)a, (Cx*)out, N, sc);
    return hipGetLastError();
}

hipError_t cd_apply_op(int dim, const void* u, const void* g, void* out, CDConst K, CDLevel L, hipStream_t s) {
    const unsigned b = nblk(ncells(dim, L.n));
    if (dim == 2) k_cd_apply<2><<<b, NT, 0, s>>>((const Cx*)u, (const Cx*)g, (Cx*)out, K, L);
    else k_cd_apply<3><<<b, NT, 0, s>>>((const Cx*)u, (const Cx*)g, (Cx*)out, K, L);
    return hipGetLastError();
}

int cd_norm_parts(int dim, int n) { return (int)nblk(ncells(dim, n)); }

hipError_t cd_norm(int dim, const void* u, const void* f, const void* g, CDConst K, CDLevel L, double* part,
                   double* norm, hipStream_t s) {
    const int np = cd_norm_parts(dim, L.n);
    if (dim == 2) k_cd_norm<2><<<np, NT, 0, s>>>((const Cx*)u, (const Cx*)f, (const Cx*)g, K, L, part);
    else k_cd_norm<3><<<np, NT, 0, s>>>((const Cx*)u, (const Cx*)f, (const Cx*)g, K, L, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_norm_finalize(part, np, np, 0, 1, norm, s);
}

}  // namespace mg
