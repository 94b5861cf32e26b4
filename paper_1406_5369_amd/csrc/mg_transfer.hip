// Residual + full-weighting restriction, interpolation + correction, coarsest solve, copies.
#include "mg_kern.h"

namespace mg {
namespace {

// ---------------------------------------------------------------------------
// Residual + full-weighting restriction (Algorithm 1, residual and restrict)
//   fc(I) = sum_delta prod_a 2^-|delta_a| / 2^d * r(2I + delta), r = f - A u
// 2D: (0.25 rC + 0.125 ((rW+rE)+(rS+rN))) + 0.0625 ((rSW+rSE)+(rNW+rNE))
// 3D: ((0.125 rC + 0.0625 faces) + 0.03125 edges) + 0.015625 corners with
//   faces = ((rW+rE)+(rS+rN))+(rB+rT), edges = (exy+exz)+eyz, each e a sum of
//   the four edge midpoints of one coordinate plane in (-,-),(+,-),(-,+),(+,+)
//   order paired as (a+b)+(c+d), corners = (z- face quad) + (z+ face quad).
// A workgroup owns CX x CY coarse nodes: fine box of (2CX+3) x (2CY+3).
// ---------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ T fw2(const T (*Rr)[BX], int ly, int lx) {
    const T edges = (Rr[ly][lx - 1] + Rr[ly][lx + 1]) + (Rr[ly - 1][lx] + Rr[ly + 1][lx]);
    const T corners = (Rr[ly - 1][lx - 1] + Rr[ly - 1][lx + 1]) + (Rr[ly + 1][lx - 1] + Rr[ly + 1][lx + 1]);
    return (T(0.25) * Rr[ly][lx] + T(0.125) * edges) + T(0.0625) * corners;
}

template <typename T>
__device__ __forceinline__ T fw3(const T (*Rb)[BX], const T (*Rc)[BX], const T (*Ra)[BX], int ly, int lx) {
    const T faces = ((Rc[ly][lx - 1] + Rc[ly][lx + 1]) + (Rc[ly - 1][lx] + Rc[ly + 1][lx])) + (Rb[ly][lx] + Ra[ly][lx]);
    const T exy = (Rc[ly - 1][lx - 1] + Rc[ly - 1][lx + 1]) + (Rc[ly + 1][lx - 1] + Rc[ly + 1][lx + 1]);
    const T exz = (Rb[ly][lx - 1] + Rb[ly][lx + 1]) + (Ra[ly][lx - 1] + Ra[ly][lx + 1]);
    const T eyz = (Rb[ly - 1][lx] + Rb[ly + 1][lx]) + (Ra[ly - 1][lx] + Ra[ly + 1][lx]);
    const T edges = (exy + exz) + eyz;
    const T cz0 = (Rb[ly - 1][lx - 1] + Rb[ly - 1][lx + 1]) + (Rb[ly + 1][lx - 1] + Rb[ly + 1][lx + 1]);
    const T cz1 = (Ra[ly - 1][lx - 1] + Ra[ly - 1][lx + 1]) + (Ra[ly + 1][lx - 1] + Ra[ly + 1][lx + 1]);
    const T corners = cz0 + cz1;
    return ((T(0.125) * Rc[ly][lx] + T(0.0625) * faces) + T(0.03125) * edges) + T(0.015625) * corners;
}

template <typename ST, bool VAR, int BY>
__global__ __launch_bounds__(NT) void k_restrict2d(const GridDesc* __restrict__ descs, int sel) {
    using T = arith_t<ST>;
    const GridDesc d = descs[blockIdx.y];
    if (d.done && *gp(d.done)) return;
    constexpr int CX = (BX - 3) / 2, CY = (BY - 3) / 2, RPT = BY / 4;
    const int nf = d.n, nc = (nf - 1) / 2 + 1;
    const int ncx = (nc - 2 + CX - 1) / CX;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int X0 = 1 + (tile % ncx) * CX, Y0 = 1 + (tile / ncx) * CY;
    const int fx0 = 2 * X0 - 2, fy0 = 2 * Y0 - 2;
    const MG_GLOBAL ST* __restrict__ u = gp((const ST*)(sel ? d.t : d.u));
    const MG_GLOBAL ST* __restrict__ f = gp((const ST*)d.f);
    const MG_GLOBAL T* __restrict__ kf = gp((const T*)d.k);
    MG_GLOBAL ST* __restrict__ fc = gp((ST*)d.fc);
    const T c = (T)d.c;
    __shared__ T U[BY][BX];
    __shared__ T Rr[BY][BX];
    __shared__ T K[VAR ? BY : 1][BX];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int gx = fx0 + lane;
    const bool lres = lane >= 1 && lane <= 2 * CX + 1;
    T fr[RPT];
#pragma unroll
    for (int m = 0; m < RPT; ++m) {
        const int ly = w + 4 * m, gy = fy0 + ly;
        const bool ing = gx < nf && gy < nf && ly <= 2 * CY + 2 && lane <= 2 * CX + 2;
        const bool inn = gx >= 1 && gx <= nf - 2 && gy >= 1 && gy <= nf - 2;
        const size_t p = (size_t)gy * nf + gx;
        U[ly][lane] = ing ? (T)u[p] : T(0);
        if constexpr (VAR) K[ly][lane] = ing ? kf[p] : T(1);
        fr[m] = (inn && lres && ly >= 1 && ly <= 2 * CY + 1) ? (T)f[p] : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < RPT; ++m) {
        const int ly = w + 4 * m, gy = fy0 + ly;
        if (lres && ly >= 1 && ly <= 2 * CY + 1) {
            const bool inn = gx >= 1 && gx <= nf - 2 && gy >= 1 && gy <= nf - 2;
            T ds;
            Rr[ly][lane] = inn ? lds_res2<T, VAR>(U, K, ly, lane, fr[m], c, ds) : T(0);
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < CX * CY; t += NT) {
        const int X = X0 + t % CX, Y = Y0 + t / CX;
        if (X <= nc - 2 && Y <= nc - 2) fc[(size_t)Y * nc + X] = (ST)fw2<T>(Rr, 2 * (Y - Y0) + 2, 2 * (X - X0) + 2);
    }
}

// 3D: marching over fine planes; step m publishes u plane m, computes the
// residual of plane m-1 and, once planes 2K-1..2K+1 are in the residual ring,
// the coarse plane K.
template <typename ST, bool VAR, int BY>
__global__ __launch_bounds__(NT) void k_restrict3d(const GridDesc* __restrict__ descs, int sel, int zchunk) {
    using T = arith_t<ST>;
    const GridDesc d = descs[blockIdx.y];
    if (d.done && *gp(d.done)) return;
    constexpr int CX = (BX - 3) / 2, CY = (BY - 3) / 2, RPT = BY / 4;
    const int nf = d.n, nc = (nf - 1) / 2 + 1;
    const int ncx = (nc - 2 + CX - 1) / CX, ncy = (nc - 2 + CY - 1) / CY;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int tx = tile % ncx, t2 = tile / ncx, ty = t2 % ncy, tz = t2 / ncy;
    const int X0 = 1 + tx * CX, Y0 = 1 + ty * CY, Z0 = 1 + tz * zchunk, Z1 = min(Z0 + zchunk, nc - 1);
    const int fx0 = 2 * X0 - 2, fy0 = 2 * Y0 - 2;
    const MG_GLOBAL ST* __restrict__ u = gp((const ST*)(sel ? d.t : d.u));
    const MG_GLOBAL ST* __restrict__ f = gp((const ST*)d.f);
    const MG_GLOBAL T* __restrict__ kf = gp((const T*)d.k);
    MG_GLOBAL ST* __restrict__ fc = gp((ST*)d.fc);
    const T c = (T)d.c;
    __shared__ T U[3][BY][BX];
    __shared__ T Rr[3][BY][BX];
    __shared__ T K[VAR ? 3 : 1][BY][BX];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int gx = fx0 + lane;
    const bool lres = lane >= 1 && lane <= 2 * CX + 1;
    const bool colg = gx < nf && lane <= 2 * CX + 2, coli = gx >= 1 && gx <= nf - 2;
    const size_t pl = (size_t)nf * nf;
    const int mstart = 2 * Z0 - 2, mend = 2 * Z1;
    T un[RPT], kn[RPT];
    T fr[2][RPT];
    // unconditional loads from clamped addresses, values selected afterwards
    auto issue_u = [&](int z) {
        const int zc = min(z, nf - 1), xc = min(gx, nf - 1);
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            const int ly = w + 4 * m, gy = fy0 + ly;
            const bool ing = colg && gy < nf && ly <= 2 * CY + 2 && z < nf;
            const size_t p = (size_t)zc * pl + (size_t)min(gy, nf - 1) * nf + xc;
            const T v = u[p];
            un[m] = ing ? v : T(0);
            if constexpr (VAR) {
                const T kv = kf[p];
                kn[m] = ing ? kv : T(1);
            }
        }
    };
    auto issue_f = [&](int z, T (&dst)[RPT]) {
        const bool zin = z >= 1 && z <= nf - 2;
        const int zc = min(z, nf - 1), xc = min(gx, nf - 1);
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            const int ly = w + 4 * m, gy = fy0 + ly;
            const bool inn = zin && coli && gy >= 1 && gy <= nf - 2 && lres && ly >= 1 && ly <= 2 * CY + 1;
            const T v = f[(size_t)zc * pl + (size_t)min(gy, nf - 1) * nf + xc];
            dst[m] = inn ? v : T(0);
        }
    };
    auto step = [&](int mm, T (&fcur)[RPT], T (&fprev)[RPT]) {
        const int s0 = (mm - mstart) % 3, s1 = (mm - 1 - mstart + 3) % 3, s2 = (mm - 2 - mstart + 6) % 3;
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            U[s0][w + 4 * m][lane] = un[m];
            if constexpr (VAR) K[s0][w + 4 * m][lane] = kn[m];
        }
        issue_f(mm, fcur);
        if (mm + 1 <= mend) issue_u(mm + 1);
        __syncthreads();
        const int rp = mm - 1;  // residual plane
        if (rp >= mstart + 1) {
            const bool zin = rp >= 1 && rp <= nf - 2;
#pragma unroll
            for (int m = 0; m < RPT; ++m) {
                const int ly = w + 4 * m, gy = fy0 + ly;
                if (lres && ly >= 1 && ly <= 2 * CY + 1) {
                    const bool inn = zin && coli && gy >= 1 && gy <= nf - 2;
                    T ds;
                    Rr[s1][ly][lane] =
                        inn ? lds_res3<T, VAR>(U[s2], U[s1], U[s0], K[s2], K[s1], K[s0], ly, lane, fprev[m], c, ds)
                            : T(0);
                }
            }
        }
        __syncthreads();
        if (((rp & 1) == 1) && rp >= 2 * Z0 + 1) {  // rp = 2K+1: planes 2K-1..2K+1 ready
            const int Kz = (rp - 1) / 2;
            const int sb = (rp - 2 - mstart + 6) % 3, sc = (rp - 1 - mstart + 3) % 3;  // planes 2K-1, 2K
            for (int t = threadIdx.x; t < CX * CY; t += NT) {
                const int X = X0 + t % CX, Y = Y0 + t / CX;
                if (X <= nc - 2 && Y <= nc - 2)
                    fc[((size_t)Kz * nc + Y) * nc + X] = (ST)fw3<T>(Rr[sb], Rr[sc], Rr[s1], 2 * (Y - Y0) + 2,
                                                                   2 * (X - X0) + 2);
            }
        }
    };
    int mm = mstart;
    issue_u(mm);
    for (; mm + 1 <= mend; mm += 2) {
        step(mm, fr[0], fr[1]);
        step(mm + 1, fr[1], fr[0]);
    }
    if (mm <= mend) step(mm, fr[0], fr[1]);
}

// ---------------------------------------------------------------------------
// Last pre-smoothing sweep fused with the residual and full weighting
// (Algorithm 1: presmoothing, residual, restriction), 3D Laplacian, red-black
// Gauss-Seidel with red first.  A workgroup owns CX x CY coarse nodes of a
// chunk of zc coarse planes and the fine nodes of their cells (fine x in
// [2X0-1, 2X0+2CX-1), likewise y and z).  On a fine box of (2CX+7) x (2CY+7)
// nodes it relaxes red on the box minus one ring, black on the box minus two
// rings (the final values; the owned ones are written out), forms the
// residual of the final values on the box minus three rings and full
// weighting at its coarse nodes.  The march along z lags: plane kk enters,
// red on kk-1, black on kk-2, residual on kk-3, coarse plane (kk-4)/2.  The
// colour updates are in place in an LDS ring of five planes (a colour reads
// only the other colour), with rings of three residual planes and four
// right-hand-side planes.  Every value is the one the separate sweep and
// restriction compute, by the same expressions.
// ---------------------------------------------------------------------------
template <typename ST, int BY>
__global__ __launch_bounds__(NT) void k_smooth_restrict3d(const GridDesc* __restrict__ descs, int arg, int zc) {
    using T = arith_t<ST>;
    constexpr int CX = 28, CY = (BY - 7) / 2, RPT = BY / 4;
    static_assert(2 * CX + 7 <= BX && 2 * CY + 7 <= BY && RPT * 4 == BY, "box fits the tile");
    const GridDesc d = descs[blockIdx.y];
    if (d.done && *gp(d.done)) return;
    const int nf = d.n, nc = (nf - 1) / 2 + 1;
    const int ncx = (nc - 1 + CX - 1) / CX, ncy = (nc - 1 + CY - 1) / CY;
    const int tile = sweep_tile(arg, blockIdx.x, gridDim.x);
    const int tx = tile % ncx, t2 = tile / ncx, ty = t2 % ncy, tz = t2 / ncy;
    const int X0 = 1 + tx * CX, Y0 = 1 + ty * CY, Z0 = 1 + tz * zc, Z1 = min(Z0 + zc, nc);
    const int fx0 = 2 * X0 - 4, fy0 = 2 * Y0 - 4;  // fine position of lane 0, row 0
    const int za = 2 * Z0 - 1, zb = 2 * Z1 - 1;     // owned fine planes [za, zb); residual on [za, zb]
    const int kstart = za - 3, kend = zb + 3;
    const MG_GLOBAL ST* __restrict__ uin = gp((const ST*)((arg & 1) ? d.t : d.u));
    MG_GLOBAL ST* __restrict__ uout = gp((ST*)((arg & 1) ? d.u : d.t));
    const MG_GLOBAL ST* __restrict__ f = gp((const ST*)d.f);
    MG_GLOBAL ST* __restrict__ fc = gp((ST*)d.fc);
    const T c = (T)d.c, wd = (T)d.wd, om = (T)d.omega;
    __shared__ T U[5][BY][BX];    // planes kk (entered), kk-1 (red done), kk-2 .. kk-4 (final)
    __shared__ T F[4][BY][BX];    // right-hand side of planes kk .. kk-3
    __shared__ T RS[3][BY][BX];   // residual of planes kk-3 .. kk-5
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int gx = fx0 + lane;
    const bool xin = gx >= 1 && gx <= nf - 2;
    const unsigned xb = (unsigned)min(max(gx, 0), nf - 1) * (unsigned)sizeof(ST);
    const size_t pl = (size_t)nf * nf;
    T un[RPT], fn[RPT];
    auto issue = [&](int z) {
        const size_t zoff = (size_t)min(max(z, 0), nf - 1) * pl;
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            const int gy = fy0 + w + 4 * m;
            const size_t roff = zoff + (size_t)min(max(gy, 0), nf - 1) * nf;
            un[m] = (T)ld_off(uin + roff, xb);
            fn[m] = (T)ld_off(f + roff, xb);
        }
    };
    auto inner = [&](int gy, int z) { return xin && gy >= 1 && gy <= nf - 2 && z >= 1 && z <= nf - 2; };
    // residual at (ly, lane) of plane slot sc with the planes below / above
    auto res_at = [&](int sb, int sc, int sa, int sf, int ly) {
        return res_lap3(U[sc][ly][lane], U[sc][ly][lane - 1], U[sc][ly][lane + 1], U[sc][ly - 1][lane],
                        U[sc][ly + 1][lane], U[sb][ly][lane], U[sa][ly][lane], F[sf][ly][lane], c);
    };
    issue(kstart);
    for (int kk = kstart; kk <= kend; ++kk) {
        const int q = kk - kstart;
        const int u0 = q % 5, u1 = (q + 4) % 5, u2 = (q + 3) % 5, u3 = (q + 2) % 5, u4 = (q + 1) % 5;
        const int f0 = q % 4, f1 = (q + 3) % 4, f2 = (q + 2) % 4, f3 = (q + 1) % 4;
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            U[u0][w + 4 * m][lane] = un[m];
            F[f0][w + 4 * m][lane] = fn[m];
        }
        if (kk < kend) issue(kk + 1);
        __syncthreads();
        // red on plane kk-1 (box minus one ring)
        const int zr = kk - 1;
        if (zr >= kstart + 1) {
#pragma unroll
            for (int m = 0; m < RPT; ++m) {
                const int ly = w + 4 * m, gy = fy0 + ly;
                if (lane >= 1 && lane <= 2 * CX + 5 && ly >= 1 && ly <= 2 * CY + 5 && inner(gy, zr) &&
                    ((gx + gy + zr) & 1) == 0) {
                    const T r = res_at(u2, u1, u0, f1, ly);
                    U[u1][ly][lane] = stored<ST>(relax<T, false>(U[u1][ly][lane], r, T(0), c, wd, om));
                }
            }
        }
        __syncthreads();
        // black on plane kk-2 (box minus two rings); write the owned final values
        const int zk = kk - 2;
        if (zk >= kstart + 2) {
#pragma unroll
            for (int m = 0; m < RPT; ++m) {
                const int ly = w + 4 * m, gy = fy0 + ly;
                const bool in = inner(gy, zk);
                if (lane >= 2 && lane <= 2 * CX + 4 && ly >= 2 && ly <= 2 * CY + 4 && in &&
                    ((gx + gy + zk) & 1) == 1) {
                    const T r = res_at(u3, u2, u1, f2, ly);
                    U[u2][ly][lane] = stored<ST>(relax<T, false>(U[u2][ly][lane], r, T(0), c, wd, om));
                }
                if (in && lane >= 3 && lane < 2 * CX + 3 && ly >= 3 && ly < 2 * CY + 3 && zk >= za && zk < zb)
                    st_off(uout + (size_t)zk * pl + (size_t)gy * nf, xb, (ST)U[u2][ly][lane]);
            }
        }
        __syncthreads();
        // residual of the final values on plane kk-3 (box minus three rings)
        const int zs = kk - 3;
        const int r0 = q % 3, r1 = (q + 2) % 3, r2 = (q + 1) % 3;  // slots of planes kk-3, kk-4, kk-5
        if (zs >= za && zs <= zb) {
#pragma unroll
            for (int m = 0; m < RPT; ++m) {
                const int ly = w + 4 * m, gy = fy0 + ly;
                if (lane >= 3 && lane <= 2 * CX + 3 && ly >= 3 && ly <= 2 * CY + 3)
                    RS[r0][ly][lane] = inner(gy, zs) ? res_at(u4, u3, u2, f3, ly) : T(0);
            }
        }
        __syncthreads();
        // full weighting of coarse plane K with 2K + 1 = kk - 3
        if ((zs & 1) == 1 && zs >= za + 2 && zs <= zb) {
            const int Kz = (zs - 1) / 2;
            if (Kz <= nc - 2) {
                for (int t = threadIdx.x; t < CX * CY; t += NT) {
                    const int X = X0 + t % CX, Y = Y0 + t / CX;
                    if (X <= nc - 2 && Y <= nc - 2)
                        fc[((size_t)Kz * nc + Y) * nc + X] =
                            (ST)fw3<T>(RS[r2], RS[r1], RS[r0], 2 * (Y - Y0) + 4, 2 * (X - X0) + 4);
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Prolongation + correction u += P uc on inner fine nodes (used when no
// post-smoothing sweep can absorb it), coarsest solve, copies.
// ---------------------------------------------------------------------------

// One wavefront per fine row (j, k); the parities of j and k are uniform per
// wave, so only the x parity varies across lanes.  The sum is formed along x,
// then y, then z, and scaled by 1/2 per odd axis, which is the order of the
// bilinear / trilinear formulas (odd axes taken in x, y, z order).
template <typename ST, int DIM>
__global__ __launch_bounds__(NT) void k_prolong(const GridDesc* __restrict__ descs, int sel) {
    using T = arith_t<ST>;
    const GridDesc d = descs[blockIdx.y];
    if (d.done && *gp(d.done)) return;
    const int n = d.n, nc = (n - 1) / 2 + 1, m = n - 2;
    const int row = blockIdx.x * (NT / 64) + (threadIdx.x >> 6);
    const int nrows = DIM == 2 ? m : m * m;
    if (row >= nrows) return;
    const int j = 1 + row % m, k = DIM == 2 ? 0 : 1 + row / m;
    const int oj = j & 1, ok = k & 1;
    MG_GLOBAL ST* __restrict__ u = gp((ST*)(sel ? d.t : d.u)) + ((size_t)k * n + j) * n;
    const MG_GLOBAL ST* __restrict__ ec = gp((const ST*)d.uc);
    const MG_GLOBAL ST* __restrict__ q00 = ec + ((size_t)(k >> 1) * nc + (j >> 1)) * nc;  // rows (J0, K0)
    const MG_GLOBAL ST* __restrict__ q10 = q00 + (size_t)oj * nc;                      // (J1, K0)
    const MG_GLOBAL ST* __restrict__ q01 = q00 + (size_t)ok * nc * nc;                 // (J0, K1)
    const MG_GLOBAL ST* __restrict__ q11 = q01 + (size_t)oj * nc;                      // (J1, K1)
    const int lane = threadIdx.x & 63;
    for (int i = 1 + lane; i <= m; i += 64) {
        const int oi = i & 1, i0 = i >> 1, i1 = i0 + oi;
        const T a0 = q00[i0], a1 = q00[i1];
        T sy0 = oi ? a0 + a1 : a0;
        if (oj) {
            const T b0 = q10[i0], b1 = q10[i1];
            sy0 = sy0 + (oi ? b0 + b1 : b0);
        }
        T s = sy0;
        if (DIM == 3 && ok) {
            const T c0 = q01[i0], c1 = q01[i1];
            T sy1 = oi ? c0 + c1 : c0;
            if (oj) {
                const T d0 = q11[i0], d1 = q11[i1];
                sy1 = sy1 + (oi ? d0 + d1 : d0);
            }
            s = s + sy1;
        }
        const int nodd = oi + oj + ok;
        const T corr = nodd == 0 ? s : (nodd == 1 ? T(0.5) * s : (nodd == 2 ? T(0.25) * s : T(0.125) * s));
        u[i] = (ST)((T)u[i] + corr);
    }
}

// n = 3: one unknown, u = f / diag (diag = c*2d, or c*dsum).
template <typename ST, int DIM, bool VAR>
__global__ void k_coarsest(const GridDesc* __restrict__ descs) {
    using T = arith_t<ST>;
    const GridDesc d = descs[blockIdx.x];
    if (threadIdx.x != 0 || (d.done && *gp(d.done))) return;
    const int p = DIM == 2 ? 4 : 13;
    MG_GLOBAL ST* u = gp((ST*)d.u);
    const MG_GLOBAL ST* f = gp((const ST*)d.f);
    const T c = (T)d.c;
    T diag;
    if constexpr (VAR) {
        const MG_GLOBAL T* k = gp((const T*)d.k);
        const T kC = k[p];
        const int sy = 3, sz = 9;
        const T kxW = kface(k[p - 1], kC), kxC = kface(kC, k[p + 1]);
        const T kyS = kface(k[p - sy], kC), kyC = kface(kC, k[p + sy]);
        T dsum;
        if (DIM == 2) {
            dsum = (kxW + kxC) + (kyS + kyC);
        } else {
            const T kzB = kface(k[p - sz], kC), kzC = kface(kC, k[p + sz]);
            dsum = ((kxW + kxC) + (kyS + kyC)) + (kzB + kzC);
        }
        diag = c * dsum;
    } else {
        diag = c * (DIM == 2 ? T(4) : T(6));
    }
    u[p] = (ST)((T)f[p] / diag);
}

template <typename T>
__global__ __launch_bounds__(NT) void k_copy_t_to_u(const GridDesc* __restrict__ descs, size_t total) {
    const GridDesc d = descs[blockIdx.y];
    if (d.done && *gp(d.done)) return;
    MG_GLOBAL T* __restrict__ u = gp((T*)d.u);
    const MG_GLOBAL T* __restrict__ t = gp((const T*)d.t);
    for (size_t q = (size_t)blockIdx.x * NT + threadIdx.x; q < total; q += (size_t)gridDim.x * NT) u[q] = t[q];
}

template <typename T>
__global__ __launch_bounds__(NT) void k_zero_u(const GridDesc* __restrict__ descs, size_t total) {
    const GridDesc d = descs[blockIdx.y];
    if (d.done && *gp(d.done)) return;
    MG_GLOBAL T* __restrict__ u = gp((T*)d.u);
    for (size_t q = (size_t)blockIdx.x * NT + threadIdx.x; q < total; q += (size_t)gridDim.x * NT) u[q] = (T)0;
}

__global__ __launch_bounds__(NT) void k_copy_bytes(uint4* __restrict__ dst, const uint4* __restrict__ src,
                                                   size_t n16) {
    const size_t q = (size_t)blockIdx.x * NT + threadIdx.x;  // one 16-byte element per thread
    if (q < n16) dst[q] = src[q];
}

}  // namespace

int smooth_tiles(int dim, int sm, int n, TileCfg cfg) {
    const int H = sm == SM_RBGS ? 2 : 1;
    const int TX = BX - 2 * H, TY = cfg.by - 2 * H;
    const int m = n - 2;
    if (dim == 2) return cdiv(m, TX) * cdiv(m, TY);
    return cdiv(m, TX) * cdiv(m, TY) * nzchunks(m, cfg.zchunk);
}

// Tiles of the two fused pre-smoothing sweeps from a zero iterate: (64 - 6) x
// (by - 6) nodes per workgroup times z-chunks
int smooth2_tiles(int n, TileCfg cfg) {
    const int m = n - 2;
    return cdiv(m, BX - 6) * cdiv(m, cfg.by - 6) * nzchunks(m, cfg.zchunk);
}

// Tiles of the fused kernel: coarse nodes per workgroup 28 x (BY-7)/2 times zc planes
int smooth_restrict_tiles(int nf, TileCfg cfg) {
    const int nc = (nf - 1) / 2 + 1, CX = 28, CY = (cfg.by - 7) / 2;
    return cdiv(nc - 1, CX) * cdiv(nc - 1, CY) * cdiv(nc - 1, cfg.zchunk);
}

template <typename T>
hipError_t launch_smooth_restrict3d(const GridDesc* d, int ninst, int nf, int sel, TileCfg cfg, hipStream_t s) {
    if constexpr (sizeof(T) == 8) {
        return hipErrorInvalidValue;  // the LDS rings hold FP32 values (FP64 would need 96 KB)
    } else {
        if (nf < 5 || ninst <= 0 || cfg.zchunk < 1 || cfg.by != 16) return hipErrorInvalidValue;
        const dim3 grid(smooth_restrict_tiles(nf, cfg), ninst);
        const int arg = (sel & 1) | (cfg.order == 1 ? 2 : 0);
        k_smooth_restrict3d<T, 16><<<grid, NT, 0, s>>>(d, arg, cfg.zchunk);
        return hipGetLastError();
    }
}

int restrict_tiles(int dim, int nf, TileCfg cfg) {
    const int CX = (BX - 3) / 2, CY = (cfg.by - 3) / 2;
    const int mc = (nf - 1) / 2 + 1 - 2;
    if (dim == 2) return cdiv(mc, CX) * cdiv(mc, CY);
    return cdiv(mc, CX) * cdiv(mc, CY) * nzchunks(mc, cfg.zchunk);
}

int norm_tiles(int dim, int n, TileCfg cfg) {
    const int TX = cfg.xp == 2 ? 2 * BX : BX - 2, TY = cfg.by - 2, m = n - 2;
    // 2D with two nodes per lane: each of the four wavefronts of a workgroup
    // marches its own chunk of cfg.zchunk rows
    if (dim == 2 && cfg.xp == 2) return cdiv(m, TX) * cdiv(cdiv(m, cfg.zchunk), 4);
    if (dim == 2) return cdiv(m, TX) * cdiv(m, TY);
    return cdiv(m, TX) * cdiv(m, TY) * nzchunks(m, cfg.zchunk);
}

template <typename T>
hipError_t launch_restrict(int dim, bool var, const GridDesc* d, int ninst, int nf, int sel, TileCfg cfg,
                           hipStream_t s) {
    if (nf < 5 || ninst <= 0) return hipErrorInvalidValue;
    const dim3 grid(restrict_tiles(dim, nf, cfg), ninst);
    if constexpr (sizeof(T) == 2) {  // binary16 storage: Laplacian only
        if (dim == 2) {
            MG_BY_SWITCH(cfg.by, (k_restrict2d<T, false, BY><<<grid, NT, 0, s>>>(d, sel)))
        } else {
            MG_BY_SWITCH(cfg.by, (k_restrict3d<T, false, BY><<<grid, NT, 0, s>>>(d, sel, cfg.zchunk)))
        }
        return var ? hipErrorInvalidValue : hipGetLastError();
    }
    if (dim == 2) {
        if (var) {
            MG_BY_SWITCH(cfg.by, (k_restrict2d<T, true, BY><<<grid, NT, 0, s>>>(d, sel)))
        } else {
            MG_BY_SWITCH(cfg.by, (k_restrict2d<T, false, BY><<<grid, NT, 0, s>>>(d, sel)))
        }
    } else {
        if (var) {
            MG_BY_SWITCH(cfg.by, (k_restrict3d<T, true, BY><<<grid, NT, 0, s>>>(d, sel, cfg.zchunk)))
        } else {
            MG_BY_SWITCH(cfg.by, (k_restrict3d<T, false, BY><<<grid, NT, 0, s>>>(d, sel, cfg.zchunk)))
        }
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong(int dim, const GridDesc* d, int ninst, int nf, int sel, hipStream_t s) {
    const int m = nf - 2;
    const int rows = dim == 2 ? m : m * m;
    const dim3 grid(cdiv(rows, NT / 64), ninst);
    if (dim == 2) k_prolong<T, 2><<<grid, NT, 0, s>>>(d, sel);
    else k_prolong<T, 3><<<grid, NT, 0, s>>>(d, sel);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_coarsest(int dim, bool var, const GridDesc* d, int ninst, hipStream_t s) {
    if constexpr (sizeof(T) == 2) {  // binary16 storage: Laplacian only
        if (var) return hipErrorInvalidValue;
        if (dim == 2) k_coarsest<T, 2, false><<<ninst, 64, 0, s>>>(d);
        else k_coarsest<T, 3, false><<<ninst, 64, 0, s>>>(d);
        return hipGetLastError();
    }
    if (dim == 2) {
        if (var) k_coarsest<T, 2, true><<<ninst, 64, 0, s>>>(d);
        else k_coarsest<T, 2, false><<<ninst, 64, 0, s>>>(d);
    } else {
        if (var) k_coarsest<T, 3, true><<<ninst, 64, 0, s>>>(d);
        else k_coarsest<T, 3, false><<<ninst, 64, 0, s>>>(d);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_copy_t_to_u(int dim, const GridDesc* d, int ninst, int n, hipStream_t s) {
    const size_t total = dim == 2 ? (size_t)n * n : (size_t)n * n * n;
    const int blocks = (int)std::min<size_t>((total + NT - 1) / NT, 4096);
    k_copy_t_to_u<T><<<dim3(blocks, ninst), NT, 0, s>>>(d, total);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_zero_u(int dim, const GridDesc* d, int ninst, int n, hipStream_t s) {
    const size_t total = dim == 2 ? (size_t)n * n : (size_t)n * n * n;
    const int blocks = (int)std::min<size_t>((total + NT - 1) / NT, 4096);
    k_zero_u<T><<<dim3(blocks, ninst), NT, 0, s>>>(d, total);
    return hipGetLastError();
}

hipError_t launch_copy_bytes(void* dst, const void* src, size_t bytes, hipStream_t s) {
    if (bytes % 16 != 0) return hipErrorInvalidValue;
    const size_t n16 = bytes / 16;
    const size_t blocks = (n16 + NT - 1) / NT;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    if (blocks) k_copy_bytes<<<(unsigned)blocks, NT, 0, s>>>((uint4*)dst, (const uint4*)src, n16);
    return hipGetLastError();
}

#define MG_INST(T)                                                                                              \
    template hipError_t launch_restrict<T>(int, bool, const GridDesc*, int, int, int, TileCfg, hipStream_t);    \
    template hipError_t launch_prolong<T>(int, const GridDesc*, int, int, int, hipStream_t);                    \
    template hipError_t launch_coarsest<T>(int, bool, const GridDesc*, int, hipStream_t);                       \
    template hipError_t launch_copy_t_to_u<T>(int, const GridDesc*, int, int, hipStream_t);                     \
    template hipError_t launch_zero_u<T>(int, const GridDesc*, int, int, hipStream_t);                       \
    template hipError_t launch_smooth_restrict3d<T>(const GridDesc*, int, int, int, TileCfg, hipStream_t);
MG_INST(double)
MG_INST(float)
MG_INST(half_t)
#undef MG_INST

}  // namespace mg
