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
// ((W+E)+(S+N))+(B+T); a boundary face contributes zeros).  up, gq0: u and g
// of cell p; gof(q, uq): g of neighbour q (from an array or formed from uq).
template <int DIM, typename GOF>
__device__ __forceinline__ void cd_faces_with(const MG_GLOBAL Cx* u, int n, int i, int j, int k, size_t p, Cx up,
                                              Cx gq0, GOF gof, Cx& F, Cx& S) {
    const Cx zero{0.0, 0.0};
    auto face = [&](bool inside, size_t q, Cx& t, Cx& gf) {
        if (!inside) {
            t = zero;
            gf = zero;
            return;
        }
        const Cx uq = ldc(u, q);
        const Cx gq = gof(q, uq);
        gf = Cx{0.5 * (gq0.re + gq.re), 0.5 * (gq0.im + gq.im)};
        t = cx_mul(gf, cx_sub(uq, up));
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

// the same with g of every cell read from its array
template <int DIM>
__device__ __forceinline__ void cd_faces(const MG_GLOBAL Cx* u, const MG_GLOBAL Cx* g, int n, int i, int j, int k,
                                         size_t p, Cx& F, Cx& S) {
    cd_faces_with<DIM>(u, n, i, j, k, p, ldc(u, p), ldc(g, p), [&](size_t q, Cx) { return ldc(g, q); }, F, S);
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

// One cell per thread (the small 3D levels, where a marching tile has too few
// workgroups to hide its latency), g of the pre-sweep iterate: MODE 0 a
// Jacobi sweep (out of place, every g formed from uin); MODE 1 the red colour
// in place (g formed from the cells, which are all pre-sweep during it; each
// red cell also stores its pre-sweep g for the black colour); MODE 2 the
// black colour in place (its own g formed, its red neighbours' read back).
template <int DIM, int MODE>
__global__ __launch_bounds__(NT) void k_cd_relax(const Cx* uin_, Cx* uout_, const Cx* __restrict__ f_, Cx* g_,
                                                 CDConst K, CDLevel L) {
    const int n = L.n;
    const size_t N = DIM == 2 ? (size_t)n * n : (size_t)n * n * n;
    const size_t p = (size_t)blockIdx.x * NT + threadIdx.x;
    if (p >= N) return;
    int i, j, k;
    cd_ijk<DIM>(p, n, i, j, k);
    if (MODE != 0 && ((i + j + k) & 1) != (MODE == 1 ? 0 : 1)) return;
    const MG_GLOBAL Cx* uin = gp(uin_);
    MG_GLOBAL Cx* g = gp(g_);
    const Cx up = ldc(uin, p), gq0 = cd_g(K, up);
    Cx F, S;
    cd_faces_with<DIM>(uin, n, i, j, k, p, up, gq0,
                       [&](size_t q, Cx uq) { return MODE == 2 ? ldc((const MG_GLOBAL Cx*)g, q) : cd_g(K, uq); }, F,
                       S);
    const Cx Nu{K.itau * up.re - L.c * F.re, K.itau * up.im - L.c * F.im};
    const Cx r = cx_sub(ldc(gp(f_), p), Nu);
    const Cx D{K.itau + L.c * S.re, L.c * S.im};
    if constexpr (MODE == 1) stc(g, p, gq0);
    stc(gp(uout_), p, cx_add(up, cx_scale(K.omega, cx_div(r, D))));
}

// Flux sum F of cell p as cd_faces forms it, with g of each cell formed from
// u (cd_g) instead of read from an array.
template <int DIM>
__device__ __forceinline__ Cx cd_flux_u(const MG_GLOBAL Cx* u, const CDConst& K, int n, int i, int j, int k,
                                        size_t p) {
    const Cx up = ldc(u, p), gq0 = cd_g(K, up);
    const Cx zero{0.0, 0.0};
    auto face = [&](bool inside, size_t q) {
        if (!inside) return zero;
        const Cx uq = ldc(u, q), gq = cd_g(K, uq);
        const Cx gf{0.5 * (gq0.re + gq.re), 0.5 * (gq0.im + gq.im)};
        return cx_mul(gf, cx_sub(uq, up));
    };
    Cx F = cx_add(cx_add(face(i > 0, p - 1), face(i < n - 1, p + 1)),
                  cx_add(face(j > 0, p - (size_t)n), face(j < n - 1, p + (size_t)n)));
    if constexpr (DIM == 3) {
        const size_t sz = (size_t)n * n;
        F = cx_add(F, cx_add(face(k > 0, p - sz), face(k < n - 1, p + sz)));
    }
    return F;
}

// fc = N_c(uh) + rc (in place over rc), uc = uh; g of uh formed on the fly
template <int DIM>
__global__ __launch_bounds__(NT) void k_cd_coarse_rhs(const Cx* __restrict__ uh_, Cx* __restrict__ fc_,
                                                      Cx* __restrict__ uc_, CDConst K, CDLevel L) {
    const int n = L.n;
    const size_t N = DIM == 2 ? (size_t)n * n : (size_t)n * n * n;
    const size_t p = (size_t)blockIdx.x * NT + threadIdx.x;
    if (p >= N) return;
    int i, j, k;
    cd_ijk<DIM>(p, n, i, j, k);
    const MG_GLOBAL Cx* uh = gp(uh_);
    const Cx F = cd_flux_u<DIM>(uh, K, n, i, j, k, p);
    const Cx up = ldc(uh, p);
    const Cx Nv{K.itau * up.re - L.c * F.re, K.itau * up.im - L.c * F.im};  // cd_apply's expression
    MG_GLOBAL Cx* fc = gp(fc_);
    stc(fc, p, cx_add(Nv, ldc(fc, p)));
    stc(gp(uc_), p, up);
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

// ---------------------------------------------------------------------------
// Tiled sweeps: both colours of a red-black sweep (or one Jacobi sweep) in one
// launch, the diffusivity of the pre-sweep iterate formed on the fly.  g is
// stored per cell as its real factor q = 1 / (1 + (Im u / (k theta))^2)
// (g = (cos theta q, sin theta q), the same products as cd_g), u and q of a
// box in LDS; red cells are relaxed on the box minus one ring in place (a
// colour reads only the other colour), black cells on the box minus two
// rings, and the tile is written to the output array (out of place, so a
// neighbouring tile always reads the pre-sweep iterate).  Per cell the
// arithmetic is that of the operator kernels (cd_apply), in the same order.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double cd_q(const CDConst& K, Cx u) {
    const double s = u.im / K.ktheta;
    return 1.0 / (1.0 + s * s);
}

// one face: flux term (tr, ti) and face diffusivity (gr, gi)
struct CDFace {
    double tr, ti, gr, gi;
};

// relaxation from the face sums: up + omega (f - N(u)) / D
__device__ __forceinline__ Cx cd_relax_v(const CDConst& K, double c, Cx up, Cx F, Cx S, Cx fv) {
    const Cx Nu{K.itau * up.re - c * F.re, K.itau * up.im - c * F.im};
    const Cx r = cx_sub(fv, Nu);
    const Cx D{K.itau + c * S.re, c * S.im};
    return cx_add(up, cx_scale(K.omega, cx_div(r, D)));
}

__device__ __forceinline__ Cx lds_c(const d2v& v) { return Cx{v.x, v.y}; }
__device__ __forceinline__ d2v to_v(Cx c) {
    d2v v;
    v.x = c.re;
    v.y = c.im;
    return v;
}

// The FAS correction u + (uc - uh) of the cell's parent (the expression of
// k_cd_prolong), applied by the CORR variants of the tiled sweeps (the first
// post-smoothing sweep after the coarse cycle) to every in-domain value they
// load; the other variants never read uc / uh.
struct CDCorr {
    const Cx* uc;
    const Cx* uh;
};
__device__ __forceinline__ size_t cd_parent(int n, int x, int y, int z) {
    const int nc = n >> 1;
    return ((size_t)(z >> 1) * nc + (y >> 1)) * nc + (x >> 1);
}
__device__ __forceinline__ Cx cd_corr(const CDCorr& C, Cx u, int n, int x, int y, int z) {
    if (!C.uc) return u;
    const size_t q = cd_parent(n, x, y, z);
    return cx_add(u, cx_sub(ldc(gp(C.uc), q), ldc(gp(C.uh), q)));
}

constexpr int CDB_Y = 16, CDB_Y3 = 12;  // box rows of the 2D / 3D tiles (64 lanes wide)

// One face with no domain test.  The tiled sweeps store each box cell outside
// the domain as a mirror ghost: u of the inner cell it faces (a clamped load)
// and that cell's q negated.  A boundary face then computes uq - up = +0 and
// a diffusivity 0.5 (ct q + ct (-q)) = +0 (likewise sin), so its flux and
// diffusivity terms are exactly the +0 the domain test would give (for
// finite iterates), with no selects.  Only the inner cell next to a ghost
// reads it, while its own value is still the one the ghost copied (a cell
// changes only in its own colour phase, after which no cell reads the ghost).
__device__ __forceinline__ CDFace cd_face_m(Cx up, Cx gp, Cx uq, double qq, const CDConst& K) {
    const double gqr = K.ct * qq, gqi = K.st * qq;
    const double gr = 0.5 * (gp.re + gqr), gi = 0.5 * (gp.im + gqi);
    const Cx t = cx_mul(Cx{gr, gi}, cx_sub(uq, up));
    return CDFace{t.re, t.im, gr, gi};
}

// relaxation of the cell at (ly, lx) of an LDS plane P (u) / Q (q, mirror
// ghosts outside the domain) with the z-neighbours (ub, qb below; ua, qa
// above) given; 2D: no z faces
template <int DIM, int W>
__device__ __forceinline__ Cx cd_relax_lds(const CDConst& K, double c, const d2v (*P)[W], const double (*Q)[W],
                                           int ly, int lx, Cx ub, double qb, Cx ua, double qa, Cx fv) {
    const Cx up = lds_c(P[ly][lx]);
    const double qp = Q[ly][lx];
    const Cx gpv{K.ct * qp, K.st * qp};
    const CDFace fW = cd_face_m(up, gpv, lds_c(P[ly][lx - 1]), Q[ly][lx - 1], K);
    const CDFace fE = cd_face_m(up, gpv, lds_c(P[ly][lx + 1]), Q[ly][lx + 1], K);
    const CDFace fS = cd_face_m(up, gpv, lds_c(P[ly - 1][lx]), Q[ly - 1][lx], K);
    const CDFace fN = cd_face_m(up, gpv, lds_c(P[ly + 1][lx]), Q[ly + 1][lx], K);
    // ((W + E) + (S + N)) [+ (B + T)], componentwise as cx_add
    double Fr = (fW.tr + fE.tr) + (fS.tr + fN.tr), Fi = (fW.ti + fE.ti) + (fS.ti + fN.ti);
    double Sr = (fW.gr + fE.gr) + (fS.gr + fN.gr), Si = (fW.gi + fE.gi) + (fS.gi + fN.gi);
    if constexpr (DIM == 3) {
        const CDFace fB = cd_face_m(up, gpv, ub, qb, K);
        const CDFace fT = cd_face_m(up, gpv, ua, qa, K);
        Fr = Fr + (fB.tr + fT.tr);
        Fi = Fi + (fB.ti + fT.ti);
        Sr = Sr + (fB.gr + fT.gr);
        Si = Si + (fB.gi + fT.gi);
    }
    return cd_relax_v(K, c, up, Cx{Fr, Fi}, Cx{Sr, Si}, fv);
}

// 2D Jacobi: a 64 x 16 box per workgroup, the tile (box minus one ring)
// relaxed and written out
template <bool CORR, int BY>
__global__ __launch_bounds__(NT) void k_cd_sweep2d_jac(const Cx* __restrict__ uin_, Cx* __restrict__ uout_,
                                                       const Cx* __restrict__ f_, CDConst K, CDLevel L, CDCorr C) {
    constexpr int H = 1, TX = 64 - 2 * H, TY = BY - 2 * H, RPT = BY / 4;
    __shared__ d2v Ub[BY][64];
    __shared__ double Qb[BY][64];
    const int n = L.n;
    const int ntx = (n + TX - 1) / TX;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);  // XCD bands: halo rows shared in one L2
    const int tx = tile % ntx, ty = tile / ntx;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int gx = tx * TX - H + lane;
    const bool xd = gx >= 0 && gx < n;
    const MG_GLOBAL Cx* uin = gp(uin_);
    const MG_GLOBAL Cx* f = gp(f_);
    MG_GLOBAL Cx* uout = gp(uout_);
    const Cx z0{0.0, 0.0};
#pragma unroll
    for (int m = 0; m < RPT; ++m) {
        const int ly = w + 4 * m, gy = ty * TY - H + ly;
        const bool dom = xd && gy >= 0 && gy < n;  // else a mirror ghost (clamped load, q negated)
        const int gxc = min(max(gx, 0), n - 1), gyc = min(max(gy, 0), n - 1);
        Cx u = ldc(uin, (size_t)gyc * n + gxc);
        if constexpr (CORR) u = cd_corr(C, u, n, gxc, gyc, 0);
        const double q = cd_q(K, u);
        Ub[ly][lane] = to_v(u);
        Qb[ly][lane] = dom ? q : -q;
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < RPT; ++m) {
        const int ly = w + 4 * m, gy = ty * TY - H + ly;
        if (xd && gy >= 0 && gy < n && lane >= H && lane < 64 - H && ly >= H && ly < BY - H)
            stc(uout, (size_t)gy * n + gx,
                cd_relax_lds<2, 64>(K, L.c, Ub, Qb, ly, lane, z0, 1.0, z0, 1.0,
                                    ldc(f, (size_t)gy * n + gx)));
    }
}

// 3D Jacobi: a 64 x 12 box in x-y marching along z through a chunk of zc
// planes.  Each thread keeps its own cells of the last four planes (u, q and
// f) in registers for the z faces (ring position = plane mod 4, resolved at
// compile time by unrolling four steps); the plane being relaxed is in an LDS
// ring of three planes for the x-y faces.  Step kk: plane kk enters (old u,
// its q); plane kk-1 is relaxed on the tile (box minus one ring) and written
// out.
template <int RPT, bool CORR>
struct CDSweep3J {
    static constexpr int BY = 4 * RPT, H = 1, TX = 64 - 2 * H, TY = BY - 2 * H;
    d2v (*Ub)[BY][64];
    double (*Qb)[BY][64];
    const MG_GLOBAL Cx* uin;
    const MG_GLOBAL Cx* f;
    MG_GLOBAL Cx* uout;
    CDConst K;
    CDCorr C;
    double c;
    int n, lane, w, gx, z0, z1, kstart;
    size_t pl;
    bool xd;
    int gyr[RPT];
    bool yd[RPT];
    double ure[4][RPT], uim[4][RPT], qr[4][RPT], fre[4][RPT], fim[4][RPT];
    double pur[RPT], pui[RPT], pfr[RPT], pfi[RPT];  // u and f of the next plane, loaded one step ahead
    double pcr[RPT], pci[RPT], phr[RPT], phi[RPT];  // uc and uh of the parent (CORR: the correcting sweep)

    __device__ __forceinline__ Cx U(int q, int m) const { return Cx{ure[q][m], uim[q][m]}; }
    __device__ __forceinline__ Cx Fv(int q, int m) const { return Cx{fre[q][m], fim[q][m]}; }

    // clamped addresses: cells outside the domain load the inner cell they
    // face (mirror ghosts, q negated when the plane enters)
    __device__ __forceinline__ void prefetch(int z) {
        const int zc = min(max(z, 0), n - 1);
        const size_t zoff = (size_t)zc * pl;
        const int gxc = min(max(gx, 0), n - 1);
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            const int gyc = min(max(gyr[m], 0), n - 1);
            const size_t p = zoff + (size_t)gyc * n + gxc;
            const Cx u = ldc(uin, p), fv = ldc(f, p);
            if constexpr (CORR) {
                const size_t pq = cd_parent(n, gxc, gyc, zc);
                const Cx cu = ldc(gp(C.uc), pq), hu = ldc(gp(C.uh), pq);
                pcr[m] = cu.re;
                pci[m] = cu.im;
                phr[m] = hu.re;
                phi[m] = hu.im;
            }
            pur[m] = u.re;
            pui[m] = u.im;
            pfr[m] = fv.re;
            pfi[m] = fv.im;
        }
    }

    template <int P>
    __device__ __forceinline__ void step(int kk) {
        constexpr int R0 = P, R1 = (P + 3) & 3, R2 = (P + 2) & 3, R3 = (P + 1) & 3;  // planes kk .. kk-3
        const int q = kk - kstart;
        const int s0 = q % 3, s1 = (q + 2) % 3, s2 = (q + 1) % 3;                     // LDS: kk, kk-1, kk-2
        const bool zd = kk >= 0 && kk < n;
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            const int ly = w + 4 * m;
            Cx u{pur[m], pui[m]};
            if constexpr (CORR) u = cx_add(u, cx_sub(Cx{pcr[m], pci[m]}, Cx{phr[m], phi[m]}));
            const double qq = cd_q(K, u);
            const double qv = (yd[m] && zd) ? qq : -qq;
            ure[R0][m] = u.re;
            uim[R0][m] = u.im;
            qr[R0][m] = qv;
            fre[R0][m] = pfr[m];
            fim[R0][m] = pfi[m];
            Ub[s0][ly][lane] = to_v(u);
            Qb[s0][ly][lane] = qv;
        }
        prefetch(kk + 1);  // after the last step this loads a plane nobody reads (inside the grid only)
        __syncthreads();
        const int zr = kk - 1;
        if (zr >= z0 && zr < z1) {
#pragma unroll
            for (int m = 0; m < RPT; ++m) {
                const int ly = w + 4 * m;
                if (yd[m] && lane >= 1 && lane <= 62 && ly >= 1 && ly <= BY - 2) {
                    const Cx v = cd_relax_lds<3, 64>(K, c, Ub[s1], Qb[s1], ly, lane, U(R2, m),
                                                     qr[R2][m], U(R0, m), qr[R0][m], Fv(R1, m));
                    stc(uout, (size_t)zr * pl + (size_t)gyr[m] * n + gx, v);
                }
            }
        }
        // no barrier here: the next step writes the slot of plane kk-2, whose
        // last reads (step kk-1) this step's barrier already ordered
    }

    __device__ __forceinline__ void run() {
        const int kend = z1 - 1 + H;
        int kk = kstart;
        for (; kk + 3 <= kend; kk += 4) {
            step<0>(kk);
            step<1>(kk + 1);
            step<2>(kk + 2);
            step<3>(kk + 3);
        }
        if (kk <= kend) step<0>(kk);
        if (kk + 1 <= kend) step<1>(kk + 1);
        if (kk + 2 <= kend) step<2>(kk + 2);
    }
};

template <int RPT, int MINW, bool CORR>
__global__ __launch_bounds__(NT, MINW) void k_cd_sweep3d_jac(const Cx* __restrict__ uin_, Cx* __restrict__ uout_,
                                                       const Cx* __restrict__ f_, CDConst K, CDLevel L, int zc, CDCorr C) {
    using S = CDSweep3J<RPT, CORR>;
    __shared__ d2v Ub[3][S::BY][64];
    __shared__ double Qb[3][S::BY][64];
    S s;
    s.Ub = Ub;
    s.Qb = Qb;
    s.uin = gp(uin_);
    s.f = gp(f_);
    s.uout = gp(uout_);
    s.K = K;
    s.C = C;
    s.c = L.c;
    const int n = L.n;
    s.n = n;
    const int ntx = (n + S::TX - 1) / S::TX, nty = (n + S::TY - 1) / S::TY;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);  // XCD bands: halo rows shared in one L2
    const int tx = tile % ntx, t2 = tile / ntx, ty = t2 % nty, tz = t2 / nty;
    s.z0 = tz * zc;
    s.z1 = min(s.z0 + zc, n);
    s.kstart = s.z0 - S::H;
    s.lane = threadIdx.x & 63;
    s.w = threadIdx.x >> 6;
    s.gx = tx * S::TX - S::H + s.lane;
    s.xd = s.gx >= 0 && s.gx < n;
    s.pl = (size_t)n * n;
#pragma unroll
    for (int m = 0; m < RPT; ++m) {
        s.gyr[m] = ty * S::TY - S::H + s.w + 4 * m;
        s.yd[m] = s.xd && s.gyr[m] >= 0 && s.gyr[m] < n;
#pragma unroll
        for (int q = 0; q < 4; ++q) s.ure[q][m] = s.uim[q][m] = s.fre[q][m] = s.fim[q][m] = 0.0, s.qr[q][m] = 1.0;
    }
    s.prefetch(s.kstart);
    s.run();
}

// ---------------------------------------------------------------------------
// Red-black sweeps with row pairs.  The colours alternate along x, so with
// one cell per lane half the lanes of every row idle in each half-sweep.
// Here a thread owns two vertically adjacent cells of its column (box rows
// 2p and 2p+1): exactly one of them is red (row 2p when x + y (+ z) of row 2p
// is even), so each half-sweep relaxes one cell per thread and no lane
// idles.  LDS reads and the global f load take the per-lane row; register
// values (3D z-neighbours) are selected per lane.  The arithmetic per cell is
// that of cd_relax_lds, as in the one-cell-per-lane sweeps.
// ---------------------------------------------------------------------------

// 2D: a 64 x 16 box per workgroup, row pairs p = w, w + 4 of the box; red on
// the box minus one ring in place, black on the tile, written out with the
// red cells.
template <bool CORR, int BY>
__global__ __launch_bounds__(NT) void k_cd_sweep2d_rb(const Cx* __restrict__ uin_, Cx* __restrict__ uout_,
                                                      const Cx* __restrict__ f_, CDConst K, CDLevel L, CDCorr C) {
    constexpr int H = 2, TX = 64 - 2 * H, TY = BY - 2 * H, RPT = BY / 4, NPR = BY / 8;
    __shared__ d2v Ub[BY][64];
    __shared__ double Qb[BY][64];
    const int n = L.n;
    const int ntx = (n + TX - 1) / TX;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);  // XCD bands: halo rows shared in one L2
    const int tx = tile % ntx, ty = tile / ntx;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int gx = tx * TX - H + lane;
    const bool xd = gx >= 0 && gx < n;
    const MG_GLOBAL Cx* uin = gp(uin_);
    const MG_GLOBAL Cx* f = gp(f_);
    MG_GLOBAL Cx* uout = gp(uout_);
    const Cx z0{0.0, 0.0};
#pragma unroll
    for (int m = 0; m < RPT; ++m) {
        const int ly = w + 4 * m, gy = ty * TY - H + ly;
        const bool dom = xd && gy >= 0 && gy < n;  // else a mirror ghost (clamped load, q negated)
        const int gxc = min(max(gx, 0), n - 1), gyc = min(max(gy, 0), n - 1);
        Cx u = ldc(uin, (size_t)gyc * n + gxc);
        if constexpr (CORR) u = cd_corr(C, u, n, gxc, gyc, 0);
        const double q = cd_q(K, u);
        Ub[ly][lane] = to_v(u);
        Qb[ly][lane] = dom ? q : -q;
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < NPR; ++m) {
        const int ly0 = 2 * (w + 4 * m), gy0 = ty * TY - H + ly0;
        const int s = (gx + gy0) & 1;  // red row of the pair
        const int ly = ly0 + s, gy = gy0 + s;
        if (xd && gy >= 0 && gy < n && lane >= 1 && lane <= 62 && ly >= 1 && ly <= BY - 2)
            Ub[ly][lane] = to_v(cd_relax_lds<2, 64>(K, L.c, Ub, Qb, ly, lane, z0, 1.0, z0, 1.0,
                                                    ldc(f, (size_t)gy * n + gx)));
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < NPR; ++m) {
        const int ly0 = 2 * (w + 4 * m), gy0 = ty * TY - H + ly0;
        const int b = 1 - ((gx + gy0) & 1);  // black row of the pair
        const int lyb = ly0 + b, gyb = gy0 + b;
        Cx vb = z0;
        if (xd && gyb >= 0 && gyb < n && lane >= H && lane < 64 - H && lyb >= H && lyb < BY - H)
            vb = cd_relax_lds<2, 64>(K, L.c, Ub, Qb, lyb, lane, z0, 1.0, z0, 1.0,
                                     ldc(f, (size_t)gyb * n + gx));
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int ly = ly0 + e, gy = gy0 + e;
            if (xd && gy >= 0 && gy < n && lane >= H && lane < 64 - H && ly >= H && ly < BY - H)
                stc(uout, (size_t)gy * n + gx, e == b ? vb : lds_c(Ub[ly][lane]));
        }
    }
}

// 3D: a 64 x 2NW box in x-y (NW wavefronts, wavefront w owning the row pair
// 2w, 2w+1) marching along z through a chunk of planes as CDSweep3J does:
// step kk: plane kk enters (registers and an LDS ring of four planes); red on
// plane kk-1 (box minus one ring, in place); black on plane kk-2 (the tile),
// written out with its red cells.  Each thread keeps its two cells of the
// last four planes (u, q, f) in registers for the z faces.
template <int NW, bool CORR>
struct CDSweep3RB {
    static constexpr int BY = 2 * NW, H = 2, TX = 64 - 2 * H, TY = BY - 2 * H;
    d2v (*Ub)[BY][64];
    double (*Qb)[BY][64];
    const MG_GLOBAL Cx* uin;
    const MG_GLOBAL Cx* f;
    MG_GLOBAL Cx* uout;
    CDConst K;
    CDCorr C;
    double c;
    int n, lane, w, gx, gy0, z0, z1, kstart;
    size_t pl;
    bool xd, yd[2];
    double ure[4][2], uim[4][2], qr[4][2], fre[4][2], fim[4][2];
    double pur[2], pui[2], pfr[2], pfi[2];  // u and f of the next plane, loaded one step ahead
    double pcr[2], pci[2], phr[2], phi[2];  // uc and uh of the parent (CORR: the correcting sweep)

    // clamped addresses: cells outside the domain load the inner cell they
    // face (mirror ghosts, q negated when the plane enters)
    __device__ __forceinline__ void prefetch(int z) {
        const int zc = min(max(z, 0), n - 1), gxc = min(max(gx, 0), n - 1);
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int gyc = min(max(gy0 + e, 0), n - 1);
            const size_t p = (size_t)zc * pl + (size_t)gyc * n + gxc;
            const Cx u = ldc(uin, p);
            Cx cu{0.0, 0.0}, hu{0.0, 0.0};
            if constexpr (CORR) {
                const size_t pq = cd_parent(n, gxc, gyc, zc);
                cu = ldc(gp(C.uc), pq);
                hu = ldc(gp(C.uh), pq);
            }
            const Cx fv = ldc(f, p);
            pur[e] = u.re;
            pui[e] = u.im;
            pfr[e] = fv.re;
            pfi[e] = fv.im;
            pcr[e] = cu.re;
            pci[e] = cu.im;
            phr[e] = hu.re;
            phi[e] = hu.im;
        }
    }

    // register value of ring slot R for the row chosen per lane (e = 0 / 1)
    template <int R>
    __device__ __forceinline__ Cx Usel(int e) const {
        return Cx{e ? ure[R][1] : ure[R][0], e ? uim[R][1] : uim[R][0]};
    }
    template <int R>
    __device__ __forceinline__ double Qsel(int e) const { return e ? qr[R][1] : qr[R][0]; }
    template <int R>
    __device__ __forceinline__ Cx Fsel(int e) const {
        return Cx{e ? fre[R][1] : fre[R][0], e ? fim[R][1] : fim[R][0]};
    }

    template <int P>
    __device__ __forceinline__ void step(int kk) {
        constexpr int R0 = P, R1 = (P + 3) & 3, R2 = (P + 2) & 3, R3 = (P + 1) & 3;  // planes kk .. kk-3
        const int q = kk - kstart;
        const int s0 = q & 3, s1 = (q + 3) & 3, s2 = (q + 2) & 3;  // LDS ring of four: kk, kk-1, kk-2
        const bool zd = kk >= 0 && kk < n;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int ly = 2 * w + e;
            Cx u{pur[e], pui[e]};
            if constexpr (CORR) u = cx_add(u, cx_sub(Cx{pcr[e], pci[e]}, Cx{phr[e], phi[e]}));
            const double qq = cd_q(K, u);
            const double qv = (yd[e] && zd) ? qq : -qq;
            ure[R0][e] = u.re;
            uim[R0][e] = u.im;
            qr[R0][e] = qv;
            fre[R0][e] = pfr[e];
            fim[R0][e] = pfi[e];
            Ub[s0][ly][lane] = to_v(u);
            Qb[s0][ly][lane] = qv;
        }
        prefetch(kk + 1);  // after the last step this loads a plane nobody reads (inside the grid only)
        __syncthreads();
        const int zr = kk - 1;  // red plane
        if (zr >= z0 - 1 && zr >= 0 && zr <= z1 && zr < n) {
            const int s = (gx + gy0 + zr) & 1;  // red row of the pair
            const int ly = 2 * w + s;
            if ((s ? yd[1] : yd[0]) && lane >= 1 && lane <= 62 && ly >= 1 && ly <= BY - 2) {
                const Cx v = cd_relax_lds<3, 64>(K, c, Ub[s1], Qb[s1], ly, lane, Usel<R2>(s),
                                                 Qsel<R2>(s), Usel<R0>(s), Qsel<R0>(s), Fsel<R1>(s));
                Ub[s1][ly][lane] = to_v(v);
                if (s) {
                    ure[R1][1] = v.re;
                    uim[R1][1] = v.im;
                } else {
                    ure[R1][0] = v.re;
                    uim[R1][0] = v.im;
                }
            }
        }
        __syncthreads();
        const int zb = kk - 2;  // black plane (output)
        if (zb >= z0 && zb < z1) {
            const int b = 1 - ((gx + gy0 + zb) & 1);  // black row of the pair
            const int lyb = 2 * w + b;
            Cx vb{0.0, 0.0};
            if ((b ? yd[1] : yd[0]) && lane >= 2 && lane <= 61 && lyb >= 2 && lyb <= BY - 3)
                vb = cd_relax_lds<3, 64>(K, c, Ub[s2], Qb[s2], lyb, lane, Usel<R3>(b),
                                         Qsel<R3>(b), Usel<R1>(b), Qsel<R1>(b), Fsel<R2>(b));
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int ly = 2 * w + e;
                if (yd[e] && lane >= 2 && lane <= 61 && ly >= 2 && ly <= BY - 3)
                    stc(uout, (size_t)zb * pl + (size_t)(gy0 + e) * n + gx,
                        e == b ? vb : Cx{ure[R2][e], uim[R2][e]});
            }
        }
        // no barrier here: with four slots the next step writes the slot of
        // plane kk-3 (last read by step kk-1's black half, ordered by this
        // step's barriers) and its red half changes plane kk's slot, which
        // this black half does not read
    }

    __device__ __forceinline__ void run() {
        const int kend = z1 - 1 + H;
        int kk = kstart;
        for (; kk + 3 <= kend; kk += 4) {
            step<0>(kk);
            step<1>(kk + 1);
            step<2>(kk + 2);
            step<3>(kk + 3);
        }
        if (kk <= kend) step<0>(kk);
        if (kk + 1 <= kend) step<1>(kk + 1);
        if (kk + 2 <= kend) step<2>(kk + 2);
    }
};

template <int NW, int MINW, bool CORR>
__global__ __launch_bounds__(64 * NW, MINW) void k_cd_sweep3d_rb(const Cx* __restrict__ uin_, Cx* __restrict__ uout_,
                                                           const Cx* __restrict__ f_, CDConst K, CDLevel L, int zc, CDCorr C) {
    using S = CDSweep3RB<NW, CORR>;
    __shared__ d2v Ub[4][S::BY][64];
    __shared__ double Qb[4][S::BY][64];
    S s;
    s.Ub = Ub;
    s.Qb = Qb;
    s.uin = gp(uin_);
    s.f = gp(f_);
    s.uout = gp(uout_);
    s.K = K;
    s.C = C;
    s.c = L.c;
    const int n = L.n;
    s.n = n;
    const int ntx = (n + S::TX - 1) / S::TX, nty = (n + S::TY - 1) / S::TY;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);  // XCD bands: halo rows shared in one L2
    const int tx = tile % ntx, t2 = tile / ntx, ty = t2 % nty, tz = t2 / nty;
    s.z0 = tz * zc;
    s.z1 = min(s.z0 + zc, n);
    s.kstart = s.z0 - S::H;
    s.lane = threadIdx.x & 63;
    s.w = threadIdx.x >> 6;
    s.gx = tx * S::TX - S::H + s.lane;
    s.xd = s.gx >= 0 && s.gx < n;
    s.gy0 = ty * S::TY - S::H + 2 * s.w;
    s.pl = (size_t)n * n;
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        s.yd[e] = s.xd && s.gy0 + e >= 0 && s.gy0 + e < n;
#pragma unroll
        for (int q = 0; q < 4; ++q) s.ure[q][e] = s.uim[q][e] = s.fre[q][e] = s.fim[q][e] = 0.0, s.qr[q][e] = 1.0;
    }
    s.prefetch(s.kstart);
    s.run();
}

// ---------------------------------------------------------------------------
// Residual blocks: one wavefront per coarse row (2D) or per coarse row of a
// coarse plane (3D), four consecutive coarse rows per workgroup, lane =
// coarse x.  A lane loads u of its children's fine x (2X, 2X+1) on the fine
// rows 2J-1 .. 2J+2 of its children's planes and, in 3D, on rows 2J, 2J+1 of
// planes 2K-1 and 2K+2, forms q of each value once (the diffusivity of u,
// the products of the operator kernels), and takes the x neighbours of its
// children from the adjacent lanes (the lanes at the wavefront's two ends
// load theirs).  Every fine value is loaded once per wavefront, 16 B per lane
// and load, instead of once per face that reads it, and g needs no array.
// From these the lane forms its children's residuals f - N(u), per cell in
// the order of cd_apply, and either restricts them and u (the cell-centred
// averages, (c00 + c10) + (c01 + c11) per fine plane, then the planes) or
// sums their squares (the norm).
// ---------------------------------------------------------------------------
template <int DIM, bool NORM>
__global__ __launch_bounds__(NT) void k_cd_resblk(const Cx* __restrict__ u_, const Cx* __restrict__ f_,
                                                  Cx* __restrict__ uh_, Cx* __restrict__ rc_, CDConst K, CDLevel L,
                                                  double* __restrict__ part) {
    constexpr int NP = DIM == 3 ? 4 : 1;   // planes 2K-1 .. 2K+2 (3D), the one plane (2D)
    constexpr int P0 = DIM == 3 ? 1 : 0;   // first of the children's planes
    constexpr int NPC = DIM == 3 ? 2 : 1;  // children's planes
    __shared__ double red4[4];
    const int n = L.n, nc = n / 2;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int ntx = (nc + 63) >> 6, nty = (nc + 3) >> 2;
    const int tx = (int)(blockIdx.x % (unsigned)ntx), b2 = (int)(blockIdx.x / (unsigned)ntx);
    const int J = (b2 % nty) * 4 + w, KK = DIM == 3 ? b2 / nty : 0;
    const int X = tx * 64 + lane;
    const bool live = X < nc && J < nc;  // KK < nc by the grid
    const MG_GLOBAL Cx* u = gp(u_);
    const MG_GLOBAL Cx* f = gp(f_);
    const size_t pl = (size_t)n * n;
    // clamped addresses for every lane: a neighbour outside the domain loads
    // the cell it faces (uq - up = +0, so the face's flux is the +0 the
    // domain test would give; see cd_face_m), lanes past the row the last
    // cell (their values serve only as such neighbours)
    const int xa0 = min(2 * X, n - 1), xa1 = min(2 * X + 1, n - 1);
    const int xe = lane == 0 ? max(2 * X - 1, 0) : min(2 * X + 2, n - 1);
    auto row_at = [&](int p, int r) -> size_t {
        const int y = min(max(2 * J - 1 + r, 0), n - 1);
        const int z = DIM == 3 ? min(max(2 * KK - 1 + p, 0), n - 1) : 0;
        return (size_t)z * pl + (size_t)y * n;
    };
    auto needed = [](int p, int r) { return DIM == 2 || p == 1 || p == 2 || r == 1 || r == 2; };

    Cx U[NP][4][2];
    double Q[NP][4][2];
    Cx Ue[NPC][2], Fv[NPC][2][2];
    double Qe[NPC][2];
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (needed(p, r)) {
                const size_t a = row_at(p, r);
                U[p][r][0] = ldc(u, a + (size_t)xa0);
                U[p][r][1] = ldc(u, a + (size_t)xa1);
            }
#pragma unroll
    for (int pc = 0; pc < NPC; ++pc)
#pragma unroll
        for (int rc = 0; rc < 2; ++rc) {
            const size_t a = row_at(P0 + pc, 1 + rc);
            Ue[pc][rc] = ldc(u, a + (size_t)xe);
            Fv[pc][rc][0] = ldc(f, a + (size_t)xa0);
            Fv[pc][rc][1] = ldc(f, a + (size_t)xa1);
        }
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (needed(p, r)) {
                Q[p][r][0] = cd_q(K, U[p][r][0]);
                Q[p][r][1] = cd_q(K, U[p][r][1]);
            }
#pragma unroll
    for (int pc = 0; pc < NPC; ++pc)
#pragma unroll
        for (int rc = 0; rc < 2; ++rc) Qe[pc][rc] = cd_q(K, Ue[pc][rc]);

    // residual of the child at fine (2X + e, 2J + rc, 2K + pc)
    Cx R[NPC][2][2];
#pragma unroll
    for (int pc = 0; pc < NPC; ++pc)
#pragma unroll
        for (int rc = 0; rc < 2; ++rc)
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int p = P0 + pc, r = 1 + rc;
                const Cx up = U[p][r][e];
                const double qp = Q[p][r][e];
                const Cx gpv{K.ct * qp, K.st * qp};
                Cx uw, ue;
                double qw, qe;
                if (e == 0) {
                    uw = Cx{lane_prev(U[p][r][1].re), lane_prev(U[p][r][1].im)};
                    qw = lane_prev(Q[p][r][1]);
                    if (lane == 0) {
                        uw = Ue[pc][rc];
                        qw = Qe[pc][rc];
                    }
                    ue = U[p][r][1];
                    qe = Q[p][r][1];
                } else {
                    uw = U[p][r][0];
                    qw = Q[p][r][0];
                    ue = Cx{lane_next(U[p][r][0].re), lane_next(U[p][r][0].im)};
                    qe = lane_next(Q[p][r][0]);
                    if (lane == 63) {
                        ue = Ue[pc][rc];
                        qe = Qe[pc][rc];
                    }
                }
                const CDFace fW = cd_face_m(up, gpv, uw, qw, K);
                const CDFace fE = cd_face_m(up, gpv, ue, qe, K);
                const CDFace fS = cd_face_m(up, gpv, U[p][r - 1][e], Q[p][r - 1][e], K);
                const CDFace fN = cd_face_m(up, gpv, U[p][r + 1][e], Q[p][r + 1][e], K);
                double Fr = (fW.tr + fE.tr) + (fS.tr + fN.tr), Fi = (fW.ti + fE.ti) + (fS.ti + fN.ti);
                if constexpr (DIM == 3) {
                    const CDFace fB = cd_face_m(up, gpv, U[p - 1][r][e], Q[p - 1][r][e], K);
                    const CDFace fT = cd_face_m(up, gpv, U[p + 1][r][e], Q[p + 1][r][e], K);
                    Fr = Fr + (fB.tr + fT.tr);
                    Fi = Fi + (fB.ti + fT.ti);
                }
                const Cx Nu{K.itau * up.re - L.c * Fr, K.itau * up.im - L.c * Fi};
                R[pc][rc][e] = cx_sub(Fv[pc][rc][e], Nu);
            }

    if constexpr (NORM) {
        double acc = 0.0;
#pragma unroll
        for (int pc = 0; pc < NPC; ++pc)
#pragma unroll
            for (int rc = 0; rc < 2; ++rc)
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const Cx& v = R[pc][rc][e];
                    acc += v.re * v.re + v.im * v.im;
                }
        const double s = block_sum(live ? acc : 0.0, red4);
        if (threadIdx.x == 0) part[blockIdx.x] = s;
    } else {
        if (!live) return;
        auto quad = [](const Cx (&A)[2][2]) { return cx_add(cx_add(A[0][0], A[0][1]), cx_add(A[1][0], A[1][1])); };
        Cx uq[NPC][2][2];
#pragma unroll
        for (int pc = 0; pc < NPC; ++pc)
#pragma unroll
            for (int rc = 0; rc < 2; ++rc)
#pragma unroll
                for (int e = 0; e < 2; ++e) uq[pc][rc][e] = U[P0 + pc][1 + rc][e];
        Cx rv, uv;
        if constexpr (DIM == 2) {
            rv = cx_scale(0.25, quad(R[0]));
            uv = cx_scale(0.25, quad(uq[0]));
        } else {
            rv = cx_scale(0.125, cx_add(quad(R[0]), quad(R[1])));
            uv = cx_scale(0.125, cx_add(quad(uq[0]), quad(uq[1])));
        }
        const size_t q = ((size_t)KK * nc + J) * nc + X;
        stc(gp(rc_), q, rv);
        stc(gp(uh_), q, uv);
    }
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

hipError_t cd_relax(int dim, bool jacobi, const void* uin, void* uout, const void* f, void* g, CDConst K, CDLevel L,
                    int colour, hipStream_t s) {
    if (!jacobi && colour != 0 && colour != 1) return hipErrorInvalidValue;
    const unsigned b = nblk(ncells(dim, L.n));
    auto ui = (const Cx*)uin;
    auto uo = (Cx*)uout;
    auto ff = (const Cx*)f;
    auto gg = (Cx*)g;
    const int mode = jacobi ? 0 : 1 + colour;
#define MG_CD_RELAX(D)                                                                      \
    if (mode == 0) k_cd_relax<D, 0><<<b, NT, 0, s>>>(ui, uo, ff, gg, K, L);                 \
    else if (mode == 1) k_cd_relax<D, 1><<<b, NT, 0, s>>>(ui, uo, ff, gg, K, L);            \
    else k_cd_relax<D, 2><<<b, NT, 0, s>>>(ui, uo, ff, gg, K, L);
    if (dim == 2) {
        MG_CD_RELAX(2)
    } else {
        MG_CD_RELAX(3)
    }
#undef MG_CD_RELAX
    return hipGetLastError();
}

// 3D levels from this edge on use the marching tiles (below it a march has
// too few workgroups to hide its latency and the per-cell kernels are faster)
constexpr int kCDTiled3D = 128;
// wavefronts (row pairs) per workgroup of the 3D red-black sweep
constexpr int kCDSweep3Waves = 8, kCDSweep3MinWaves = 2;
// rows per thread (box height / 4) and minimum wavefronts per SIMD of the 3D Jacobi march
constexpr int kCDJacRows = 3, kCDJacMinWaves = 2;
bool cd_tiled(int dim, int n) { return dim == 2 || n >= kCDTiled3D; }
bool cd_sweep_corrects(int dim, bool jacobi, int n) { return cd_tiled(dim, n); }

hipError_t cd_sweep(int dim, bool jacobi, const void* uin, void* uout, const void* f, CDConst K, CDLevel L,
                    hipStream_t s, const void* uc, const void* uh) {
    if ((uc == nullptr) != (uh == nullptr)) return hipErrorInvalidValue;
    const CDCorr C{(const Cx*)uc, (const Cx*)uh};
    const int n = L.n;
    auto ui = (const Cx*)uin;
    auto uo = (Cx*)uout;
    auto ff = (const Cx*)f;
    if (dim == 2) {
        const int H = jacobi ? 1 : 2;
        constexpr int BY = CDB_Y;
        const unsigned b = (unsigned)(((n + 64 - 2 * H - 1) / (64 - 2 * H)) * ((n + BY - 2 * H - 1) / (BY - 2 * H)));
        if (jacobi) {
            if (C.uc) k_cd_sweep2d_jac<true, BY><<<b, NT, 0, s>>>(ui, uo, ff, K, L, C);
            else k_cd_sweep2d_jac<false, BY><<<b, NT, 0, s>>>(ui, uo, ff, K, L, C);
        } else {
            if (C.uc) k_cd_sweep2d_rb<true, BY><<<b, NT, 0, s>>>(ui, uo, ff, K, L, C);
            else k_cd_sweep2d_rb<false, BY><<<b, NT, 0, s>>>(ui, uo, ff, K, L, C);
        }
    } else {
        if (n < kCDTiled3D) return hipErrorInvalidValue;  // small levels take the per-cell kernels
        auto cdiv = [](int a, int d) { return (unsigned)((a + d - 1) / d); };
        if (jacobi) {
            constexpr int zc = 8;
            if (C.uc) {  // two rows per thread: room for the correction's registers
                using S = CDSweep3J<2, true>;
                const unsigned b = cdiv(n, S::TX) * cdiv(n, S::TY) * cdiv(n, zc);
                k_cd_sweep3d_jac<2, kCDJacMinWaves, true><<<b, NT, 0, s>>>(ui, uo, ff, K, L, zc, C);
            } else {
                using S = CDSweep3J<kCDJacRows, false>;
                const unsigned b = cdiv(n, S::TX) * cdiv(n, S::TY) * cdiv(n, zc);
                k_cd_sweep3d_jac<kCDJacRows, kCDJacMinWaves, false><<<b, NT, 0, s>>>(ui, uo, ff, K, L, zc, C);
            }
        } else {
            // 16-plane chunks at 256^3; smaller levels take 8 for twice the workgroups
            constexpr int NW = kCDSweep3Waves;
            const int zc = n >= 256 ? 16 : 8;
            using S = CDSweep3RB<NW, false>;
            const unsigned b = cdiv(n, S::TX) * cdiv(n, S::TY) * cdiv(n, zc);
            if (C.uc) k_cd_sweep3d_rb<NW, kCDSweep3MinWaves, true><<<b, 64 * NW, 0, s>>>(ui, uo, ff, K, L, zc, C);
            else k_cd_sweep3d_rb<NW, kCDSweep3MinWaves, false><<<b, 64 * NW, 0, s>>>(ui, uo, ff, K, L, zc, C);
        }
    }
    return hipGetLastError();
}

static unsigned cd_resblk_blocks(int dim, int n) {
    const unsigned nc = (unsigned)(n / 2);
    const unsigned b = ((nc + 63) / 64) * ((nc + 3) / 4);
    return dim == 3 ? b * nc : b;
}

hipError_t cd_restrict(int dim, const void* u, const void* f, void* uh, void* rc, CDConst K, CDLevel L,
                       hipStream_t s) {
    if (L.n < 2) return hipErrorInvalidValue;
    const unsigned b = cd_resblk_blocks(dim, L.n);
    if (dim == 2)
        k_cd_resblk<2, false><<<b, NT, 0, s>>>((const Cx*)u, (const Cx*)f, (Cx*)uh, (Cx*)rc, K, L, nullptr);
    else
        k_cd_resblk<3, false><<<b, NT, 0, s>>>((const Cx*)u, (const Cx*)f, (Cx*)uh, (Cx*)rc, K, L, nullptr);
    return hipGetLastError();
}

hipError_t cd_coarse_rhs(int dim, const void* uh, void* fc, void* uc, CDConst K, CDLevel Lc, hipStream_t s) {
    const unsigned b = nblk(ncells(dim, Lc.n));
    if (dim == 2)
        k_cd_coarse_rhs<2><<<b, NT, 0, s>>>((const Cx*)uh, (Cx*)fc, (Cx*)uc, K, Lc);
    else
        k_cd_coarse_rhs<3><<<b, NT, 0, s>>>((const Cx*)uh, (Cx*)fc, (Cx*)uc, K, Lc);
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

int cd_norm_parts(int dim, int n) { return (int)cd_resblk_blocks(dim, n); }

hipError_t cd_norm(int dim, const void* u, const void* f, CDConst K, CDLevel L, double* part, double* norm,
                   hipStream_t s) {
    if (L.n < 2) return hipErrorInvalidValue;
    const int np = cd_norm_parts(dim, L.n);
    if (dim == 2) k_cd_resblk<2, true><<<np, NT, 0, s>>>((const Cx*)u, (const Cx*)f, nullptr, nullptr, K, L, part);
    else k_cd_resblk<3, true><<<np, NT, 0, s>>>((const Cx*)u, (const Cx*)f, nullptr, nullptr, K, L, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_norm_finalize(part, np, np, 0, 1, norm, s);
}

}  // namespace mg
