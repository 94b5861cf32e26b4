// HIP kernels of the geometric multigrid V-cycle for gfx950 (CDNA4).
//
// The method (Koestler et al., arXiv:1406.5369): node-based second-order
// finite differences (Section 2.2) on the unit square / cube with zero
// Dirichlet boundary, the recursive V-cycle of Algorithm 1 (Section 2.3) with
// omega-Jacobi or red-black Gauss-Seidel smoothing (Section 2.3 component
// list, Section 2.4 GaussSeidel), full-weighting restriction and its partner
// bi-/trilinear interpolation (Section 2.3, Section 2.4 Restrict /
// interpolatecorr), and the L2 residual of the solve loop (Section 2.4
// Application).
//
// Per-point arithmetic is written in one fixed evaluation order and the file
// is compiled without floating-point contraction, so every update rounds
// exactly like any other implementation writing the same expressions:
//   2D  r = f - c*(4 uC - ((uW+uE)+(uS+uN)))
//   3D  r = f - c*(6 uC - (((uW+uE)+(uS+uN))+(uB+uT)))
//   relaxation (Section 2.4): u = uC + wd*r, wd = omega*h^2/(2d)
//   variable coefficients: face k = ((2a)b)/(a+b) (harmonic mean),
//     dsum = ((kxW+kxC)+(kyS+kyC))[+(kzB+kzC)], t = sum of k_face*u_nb in the
//     same pairing, r = f - c*(dsum uC - t), u = uC + (omega r)/(c dsum)
//   full weighting and interpolation: see the restriction and interp helpers.
//
// Data layout: one dense array per field, x fastest, idx = (k*n + j)*n + i.
// Workgroups are 256 threads (four wave64); a workgroup owns an x-y tile and,
// in 3D, marches along z through a chunk of planes, keeping a ring of three
// planes in LDS (halo included) so each HBM value is fetched about once per
// sweep.  Red-black Gauss-Seidel is fused: the red half-sweep is computed on
// the tile plus a one-node ring (from a two-node ring of old values), the
// black half-sweep on the tile, and the result is written out-of-place to the
// ping-pong buffer, so tiles never read values another tile has updated.
#include "mg_internal.h"

#include <algorithm>

namespace mg {
namespace {

constexpr int BX = 64;   // LDS box width: one wavefront per row
constexpr int NT = 256;  // threads per workgroup

// ---------------------------------------------------------------------------
// Per-point arithmetic
// ---------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ T kface(T a, T b) {
    return ((T(2) * a) * b) / (a + b);
}

template <typename T>
__device__ __forceinline__ T res_lap2(T uC, T uW, T uE, T uS, T uN, T f, T c) {
    const T s = (uW + uE) + (uS + uN);
    return f - c * (T(4) * uC - s);
}

template <typename T>
__device__ __forceinline__ T res_lap3(T uC, T uW, T uE, T uS, T uN, T uB, T uT, T f, T c) {
    const T s = ((uW + uE) + (uS + uN)) + (uB + uT);
    return f - c * (T(6) * uC - s);
}

template <typename T>
__device__ __forceinline__ T res_var2(T uC, T uW, T uE, T uS, T uN, T kC, T kW, T kE, T kS, T kN, T f, T c,
                                      T& dsum) {
    const T kxW = kface(kW, kC), kxC = kface(kC, kE);
    const T kyS = kface(kS, kC), kyC = kface(kC, kN);
    dsum = (kxW + kxC) + (kyS + kyC);
    const T t = (kxW * uW + kxC * uE) + (kyS * uS + kyC * uN);
    return f - c * (dsum * uC - t);
}

template <typename T>
__device__ __forceinline__ T res_var3(T uC, T uW, T uE, T uS, T uN, T uB, T uT, T kC, T kW, T kE, T kS, T kN, T kB,
                                      T kT, T f, T c, T& dsum) {
    const T kxW = kface(kW, kC), kxC = kface(kC, kE);
    const T kyS = kface(kS, kC), kyC = kface(kC, kN);
    const T kzB = kface(kB, kC), kzC = kface(kC, kT);
    dsum = ((kxW + kxC) + (kyS + kyC)) + (kzB + kzC);
    const T t = ((kxW * uW + kxC * uE) + (kyS * uS + kyC * uN)) + (kzB * uB + kzC * uT);
    return f - c * (dsum * uC - t);
}

// 2D stencil evaluation on an LDS box A (and coefficient box K), centre (ly, lx).
template <typename T, bool VAR>
__device__ __forceinline__ T lds_res2(const T (*A)[BX], const T (*K)[BX], int ly, int lx, T f, T c, T& dsum) {
    if constexpr (VAR) {
        return res_var2(A[ly][lx], A[ly][lx - 1], A[ly][lx + 1], A[ly - 1][lx], A[ly + 1][lx], K[ly][lx],
                        K[ly][lx - 1], K[ly][lx + 1], K[ly - 1][lx], K[ly + 1][lx], f, c, dsum);
    } else {
        dsum = T(0);
        return res_lap2(A[ly][lx], A[ly][lx - 1], A[ly][lx + 1], A[ly - 1][lx], A[ly + 1][lx], f, c);
    }
}

// 3D: planes Ab (below, z-1), Ac (centre), Aa (above, z+1).
template <typename T, bool VAR>
__device__ __forceinline__ T lds_res3(const T (*Ab)[BX], const T (*Ac)[BX], const T (*Aa)[BX], const T (*Kb)[BX],
                                      const T (*Kc)[BX], const T (*Ka)[BX], int ly, int lx, T f, T c, T& dsum) {
    if constexpr (VAR) {
        return res_var3(Ac[ly][lx], Ac[ly][lx - 1], Ac[ly][lx + 1], Ac[ly - 1][lx], Ac[ly + 1][lx], Ab[ly][lx],
                        Aa[ly][lx], Kc[ly][lx], Kc[ly][lx - 1], Kc[ly][lx + 1], Kc[ly - 1][lx], Kc[ly + 1][lx],
                        Kb[ly][lx], Ka[ly][lx], f, c, dsum);
    } else {
        dsum = T(0);
        return res_lap3(Ac[ly][lx], Ac[ly][lx - 1], Ac[ly][lx + 1], Ac[ly - 1][lx], Ac[ly + 1][lx], Ab[ly][lx],
                        Aa[ly][lx], f, c);
    }
}

// Relaxation of Section 2.4: u + omega * diag^-1 * r.
template <typename T, bool VAR>
__device__ __forceinline__ T relax(T uC, T r, T dsum, T c, T wd, T om) {
    if constexpr (VAR) {
        return uC + (om * r) / (c * dsum);
    } else {
        return uC + wd * r;
    }
}

// Bilinear interpolation of the coarse correction at fine node (i, j):
// coincident nodes copy, edge midpoints average two, cell centres four.
template <typename T>
__device__ __forceinline__ T interp2(const T* __restrict__ e, int nc, int i, int j) {
    const T* q = e + (size_t)(j >> 1) * nc + (i >> 1);
    const int oi = i & 1, oj = j & 1;
    if (!oi && !oj) return q[0];
    if (oi && !oj) return T(0.5) * (q[0] + q[1]);
    if (!oi && oj) return T(0.5) * (q[0] + q[nc]);
    return T(0.25) * ((q[0] + q[1]) + (q[nc] + q[nc + 1]));
}

// Trilinear interpolation at fine node (i, j, k); the odd axes are taken in
// x, y, z order (s0 first, s1 second, s2 third).
template <typename T>
__device__ __forceinline__ T interp3(const T* __restrict__ e, int nc, int i, int j, int k) {
    const size_t sy = (size_t)nc, sz = (size_t)nc * nc;
    const T* q = e + (size_t)(k >> 1) * sz + (size_t)(j >> 1) * sy + (i >> 1);
    size_t s[3];
    int m = 0;
    if (i & 1) s[m++] = 1;
    if (j & 1) s[m++] = sy;
    if (k & 1) s[m++] = sz;
    if (m == 0) return q[0];
    if (m == 1) return T(0.5) * (q[0] + q[s[0]]);
    if (m == 2) return T(0.25) * ((q[0] + q[s[0]]) + (q[s[1]] + q[s[0] + s[1]]));
    return T(0.125) * (((q[0] + q[1]) + (q[sy] + q[1 + sy])) + ((q[sz] + q[1 + sz]) + (q[sy + sz] + q[1 + sy + sz])));
}

// Map the dispatch-order block id to a tile id such that the blocks that land
// on one XCD (dispatch is round-robin over the 8 XCDs) get a contiguous range
// of tiles, which share halo rows in that XCD's L2.
__device__ __forceinline__ int xcd_tile(int b, int G) {
    const int q = G >> 3, r = G & 7;
    const int x = b & 7, i = b >> 3;
    return x * q + (x < r ? x : r) + i;
}

// Deterministic workgroup sum of one double per thread (fixed shuffle order,
// then the four wave partials in order).  Result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* red4) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red4[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) s = (red4[0] + red4[1]) + (red4[2] + red4[3]);
    return s;
}

// ---------------------------------------------------------------------------
// 2D smoothing sweep (one LDS tile per workgroup, no marching)
// ---------------------------------------------------------------------------

template <typename T, int SM, bool VAR, int BY>
__global__ __launch_bounds__(NT) void k_smooth2d(const GridDesc* __restrict__ descs, int sel, int flags) {
    const GridDesc d = descs[blockIdx.y];
    if (d.done && *d.done) return;
    constexpr int H = SM == SM_RBGS ? 2 : 1;
    constexpr int TX = BX - 2 * H, TY = BY - 2 * H, RPT = BY / 4;
    const int n = d.n;
    const int ntx = (n - 2 + TX - 1) / TX;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int x0 = 1 + (tile % ntx) * TX, y0 = 1 + (tile / ntx) * TY;
    const T* __restrict__ uin = (const T*)(sel ? d.t : d.u);
    T* __restrict__ uout = (T*)(sel ? d.u : d.t);
    const T* __restrict__ f = (const T*)d.f;
    const T* __restrict__ kf = (const T*)d.k;
    const T* __restrict__ ec = (const T*)d.uc;
    const int nc = (n - 1) / 2 + 1;
    const T c = (T)d.c, wd = (T)d.wd, om = (T)d.omega;

    __shared__ T U[BY][BX];
    __shared__ T R[SM == SM_RBGS ? BY : 1][BX];
    __shared__ T K[VAR ? BY : 1][BX];

    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int gx = x0 - H + lane;
    const bool colg = gx >= 0 && gx < n, coli = gx >= 1 && gx <= n - 2;
    const bool lane1 = lane >= 1 && lane <= BX - 2;  // tile + 1 ring (RBGS) / tile (Jacobi)
    T fr[RPT];
#pragma unroll
    for (int m = 0; m < RPT; ++m) {
        const int ly = w + 4 * m, gy = y0 - H + ly;
        const bool ing = colg && gy >= 0 && gy < n;
        const bool inn = coli && gy >= 1 && gy <= n - 2;
        const size_t p = (size_t)gy * n + gx;
        T v = T(0);
        if (ing && !(flags & SWEEP_ZERO_GUESS)) v = uin[p];
        if (inn && (flags & SWEEP_PROLONG)) v = v + interp2(ec, nc, gx, gy);
        U[ly][lane] = v;
        if constexpr (VAR) K[ly][lane] = ing ? kf[p] : T(1);
        fr[m] = (inn && lane1 && ly >= 1 && ly <= BY - 2) ? f[p] : T(0);
    }
    __syncthreads();
    if constexpr (SM == SM_RBGS) {
        // red half-sweep on the tile plus a one-node ring
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            const int ly = w + 4 * m, gy = y0 - H + ly;
            if (lane1 && ly >= 1 && ly <= BY - 2) {
                const bool inn = coli && gy >= 1 && gy <= n - 2;
                T v = U[ly][lane];
                if (inn && ((gx + gy) & 1) == 0) {
                    T ds;
                    const T r = lds_res2<T, VAR>(U, K, ly, lane, fr[m], c, ds);
                    v = relax<T, VAR>(v, r, ds, c, wd, om);
                }
                R[ly][lane] = v;
            }
        }
        __syncthreads();
        // black half-sweep on the tile, written out of place
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            const int ly = w + 4 * m, gy = y0 - H + ly;
            if (lane >= 2 && lane <= BX - 3 && ly >= 2 && ly <= BY - 3 && gx <= n - 2 && gy <= n - 2) {
                T v = R[ly][lane];
                if (((gx + gy) & 1) == 1) {
                    T ds;
                    const T r = lds_res2<T, VAR>(R, K, ly, lane, fr[m], c, ds);
                    v = relax<T, VAR>(v, r, ds, c, wd, om);
                }
                uout[(size_t)gy * n + gx] = v;
            }
        }
    } else {
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            const int ly = w + 4 * m, gy = y0 - H + ly;
            if (lane1 && ly >= 1 && ly <= BY - 2 && gx <= n - 2 && gy <= n - 2) {
                T ds;
                const T r = lds_res2<T, VAR>(U, K, ly, lane, fr[m], c, ds);
                uout[(size_t)gy * n + gx] = relax<T, VAR>(U[ly][lane], r, ds, c, wd, om);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// 3D smoothing sweep: x-y tile, marching along z through a chunk of planes.
//
// RBGS step kk (plane kk enters the LDS ring):
//   A  publish old u of plane kk (prefetched one step earlier), prefetch kk+1
//   B  red relaxation of plane kk-1 on the tile + one-node ring
//   C  black relaxation of plane kk-2 on the tile, written to the output
// Jacobi step kk: A as above, B relaxes plane kk-1 on the tile.
// LDS rings are indexed by (plane - first plane) mod 3; register rings of f
// use the same index, resolved at compile time by unrolling three steps.
// ---------------------------------------------------------------------------

template <typename T, int SM, bool VAR, int BY>
struct Smooth3D {
    static constexpr int H = SM == SM_RBGS ? 2 : 1;
    static constexpr int TX = BX - 2 * H, TY = BY - 2 * H, RPT = BY / 4;

    T (*U)[BY][BX];
    T (*R)[BY][BX];
    T (*K)[BY][BX];
    const T* __restrict__ uin;
    T* __restrict__ uout;
    const T* __restrict__ f;
    const T* __restrict__ kf;
    int n, x0, y0, z0, z1, kstart, kend, flags;
    T c, wd, om;
    int lane, w, gx;
    bool colg, coli, lane1;
    T un[RPT], kn[RPT];
    T fr[3][RPT];

    __device__ __forceinline__ size_t at(int x, int y, int z) const {
        return ((size_t)z * n + y) * n + x;
    }
    __device__ __forceinline__ int gy(int m) const { return y0 - H + w + 4 * m; }

    __device__ __forceinline__ void issue_u(int z) {
        const bool zok = z >= 0 && z < n;
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            const int y = gy(m);
            const bool ing = zok && colg && y >= 0 && y < n;
            un[m] = (ing && !(flags & SWEEP_ZERO_GUESS)) ? uin[at(gx, y, z)] : T(0);
            if constexpr (VAR) kn[m] = ing ? kf[at(gx, y, z)] : T(1);
        }
    }
    __device__ __forceinline__ void issue_f(int z, T (&dst)[RPT]) {
        const bool zin = z >= 1 && z <= n - 2;
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            const int y = gy(m), ly = w + 4 * m;
            const bool inn = zin && coli && y >= 1 && y <= n - 2 && lane1 && ly >= 1 && ly <= BY - 2;
            dst[m] = inn ? f[at(gx, y, z)] : T(0);
        }
    }

    template <int P>
    __device__ __forceinline__ void step(int kk) {
        constexpr int S0 = P, S1 = (P + 2) % 3, S2 = (P + 1) % 3;  // slots of planes kk, kk-1, kk-2
        const int k4 = (kk - kstart) & 3;                            // coefficient ring (4 planes)
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            U[S0][w + 4 * m][lane] = un[m];
            if constexpr (VAR) K[k4][w + 4 * m][lane] = kn[m];
        }
        issue_f(kk, fr[S0]);
        if (kk + 1 <= kend) issue_u(kk + 1);
        __syncthreads();
        if constexpr (SM == SM_RBGS) {
            const int m1 = kk - 1;  // red plane
            if (m1 >= z0 - 1) {
                const bool zin = m1 >= 1 && m1 <= n - 2;
                const int kb = (kk - 2 - kstart) & 3, kc = (kk - 1 - kstart) & 3;
#pragma unroll
                for (int m = 0; m < RPT; ++m) {
                    const int ly = w + 4 * m, y = gy(m);
                    if (lane1 && ly >= 1 && ly <= BY - 2) {
                        T v = U[S1][ly][lane];
                        if (zin && coli && y >= 1 && y <= n - 2 && ((gx + y + m1) & 1) == 0) {
                            T ds;
                            const T r = lds_res3<T, VAR>(U[S2], U[S1], U[S0], K[kb], K[kc], K[k4], ly, lane,
                                                         fr[S1][m], c, ds);
                            v = relax<T, VAR>(v, r, ds, c, wd, om);
                        }
                        R[S1][ly][lane] = v;
                    }
                }
            }
            __syncthreads();
            const int m2 = kk - 2;  // black plane (output)
            if (m2 >= z0 && m2 < z1) {
                const int kb = (kk - 3 - kstart) & 3, kc = (kk - 2 - kstart) & 3, ka = (kk - 1 - kstart) & 3;
#pragma unroll
                for (int m = 0; m < RPT; ++m) {
                    const int ly = w + 4 * m, y = gy(m);
                    if (lane >= 2 && lane <= BX - 3 && ly >= 2 && ly <= BY - 3 && gx <= n - 2 && y <= n - 2) {
                        T v = R[S2][ly][lane];
                        if (((gx + y + m2) & 1) == 1) {
                            T ds;
                            const T r = lds_res3<T, VAR>(R[P], R[S2], R[S1], K[kb], K[kc], K[ka], ly, lane,
                                                         fr[S2][m], c, ds);
                            v = relax<T, VAR>(v, r, ds, c, wd, om);
                        }
                        uout[at(gx, y, m2)] = v;
                    }
                }
            }
            if constexpr (VAR) __syncthreads();  // K slot of plane kk-3 is rewritten next step
        } else {
            const int m1 = kk - 1;
            if (m1 >= z0 && m1 < z1) {
                const int kb = (kk - 2 - kstart) & 3, kc = (kk - 1 - kstart) & 3;
#pragma unroll
                for (int m = 0; m < RPT; ++m) {
                    const int ly = w + 4 * m, y = gy(m);
                    if (lane1 && ly >= 1 && ly <= BY - 2 && gx <= n - 2 && y <= n - 2) {
                        T ds;
                        const T r = lds_res3<T, VAR>(U[S2], U[S1], U[S0], K[kb], K[kc], K[k4], ly, lane,
                                                     fr[S1][m], c, ds);
                        uout[at(gx, y, m1)] = relax<T, VAR>(U[S1][ly][lane], r, ds, c, wd, om);
                    }
                }
            }
            __syncthreads();
        }
    }

    __device__ __forceinline__ void run() {
        int kk = kstart;
        issue_u(kk);
        for (; kk + 2 <= kend; kk += 3) {
            step<0>(kk);
            step<1>(kk + 1);
            step<2>(kk + 2);
        }
        if (kk <= kend) step<0>(kk);
        if (kk + 1 <= kend) step<1>(kk + 1);
    }
};

template <typename T, int SM, bool VAR, int BY>
__global__ __launch_bounds__(NT) void k_smooth3d(const GridDesc* __restrict__ descs, int sel, int flags,
                                                 int zchunk) {
    const GridDesc d = descs[blockIdx.y];
    if (d.done && *d.done) return;
    using S = Smooth3D<T, SM, VAR, BY>;
    __shared__ T U[3][BY][BX];
    __shared__ T R[SM == SM_RBGS ? 3 : 1][BY][BX];
    __shared__ T K[VAR ? 4 : 1][BY][BX];
    S s;
    s.U = U;
    s.R = R;
    s.K = K;
    const int n = d.n;
    const int ntx = (n - 2 + S::TX - 1) / S::TX, nty = (n - 2 + S::TY - 1) / S::TY;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int tx = tile % ntx, t2 = tile / ntx, ty = t2 % nty, tz = t2 / nty;
    s.n = n;
    s.x0 = 1 + tx * S::TX;
    s.y0 = 1 + ty * S::TY;
    s.z0 = 1 + tz * zchunk;
    s.z1 = min(s.z0 + zchunk, n - 1);
    s.kstart = s.z0 - S::H;
    s.kend = s.z1 - 1 + S::H;
    s.flags = flags;
    s.uin = (const T*)(sel ? d.t : d.u);
    s.uout = (T*)(sel ? d.u : d.t);
    s.f = (const T*)d.f;
    s.kf = (const T*)d.k;
    s.c = (T)d.c;
    s.wd = (T)d.wd;
    s.om = (T)d.omega;
    s.lane = threadIdx.x & 63;
    s.w = threadIdx.x >> 6;
    s.gx = s.x0 - S::H + s.lane;
    s.colg = s.gx >= 0 && s.gx < n;
    s.coli = s.gx >= 1 && s.gx <= n - 2;
    s.lane1 = s.lane >= 1 && s.lane <= BX - 2;
    s.run();
}

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

template <typename T, bool VAR, int BY>
__global__ __launch_bounds__(NT) void k_restrict2d(const GridDesc* __restrict__ descs, int sel) {
    const GridDesc d = descs[blockIdx.y];
    if (d.done && *d.done) return;
    constexpr int CX = (BX - 3) / 2, CY = (BY - 3) / 2, RPT = BY / 4;
    const int nf = d.n, nc = (nf - 1) / 2 + 1;
    const int ncx = (nc - 2 + CX - 1) / CX;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int X0 = 1 + (tile % ncx) * CX, Y0 = 1 + (tile / ncx) * CY;
    const int fx0 = 2 * X0 - 2, fy0 = 2 * Y0 - 2;
    const T* __restrict__ u = (const T*)(sel ? d.t : d.u);
    const T* __restrict__ f = (const T*)d.f;
    const T* __restrict__ kf = (const T*)d.k;
    T* __restrict__ fc = (T*)d.fc;
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
        U[ly][lane] = ing ? u[p] : T(0);
        if constexpr (VAR) K[ly][lane] = ing ? kf[p] : T(1);
        fr[m] = (inn && lres && ly >= 1 && ly <= 2 * CY + 1) ? f[p] : T(0);
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
        if (X <= nc - 2 && Y <= nc - 2) fc[(size_t)Y * nc + X] = fw2<T>(Rr, 2 * (Y - Y0) + 2, 2 * (X - X0) + 2);
    }
}

// 3D: marching over fine planes; step m publishes u plane m, computes the
// residual of plane m-1 and, once planes 2K-1..2K+1 are in the residual ring,
// the coarse plane K.
template <typename T, bool VAR, int BY>
__global__ __launch_bounds__(NT) void k_restrict3d(const GridDesc* __restrict__ descs, int sel, int zchunk) {
    const GridDesc d = descs[blockIdx.y];
    if (d.done && *d.done) return;
    constexpr int CX = (BX - 3) / 2, CY = (BY - 3) / 2, RPT = BY / 4;
    const int nf = d.n, nc = (nf - 1) / 2 + 1;
    const int ncx = (nc - 2 + CX - 1) / CX, ncy = (nc - 2 + CY - 1) / CY;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int tx = tile % ncx, t2 = tile / ncx, ty = t2 % ncy, tz = t2 / ncy;
    const int X0 = 1 + tx * CX, Y0 = 1 + ty * CY, Z0 = 1 + tz * zchunk, Z1 = min(Z0 + zchunk, nc - 1);
    const int fx0 = 2 * X0 - 2, fy0 = 2 * Y0 - 2;
    const T* __restrict__ u = (const T*)(sel ? d.t : d.u);
    const T* __restrict__ f = (const T*)d.f;
    const T* __restrict__ kf = (const T*)d.k;
    T* __restrict__ fc = (T*)d.fc;
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
    auto issue_u = [&](int z) {
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            const int ly = w + 4 * m, gy = fy0 + ly;
            const bool ing = colg && gy < nf && ly <= 2 * CY + 2 && z < nf;
            const size_t p = (size_t)z * pl + (size_t)gy * nf + gx;
            un[m] = ing ? u[p] : T(0);
            if constexpr (VAR) kn[m] = ing ? kf[p] : T(1);
        }
    };
    auto issue_f = [&](int z, T (&dst)[RPT]) {
        const bool zin = z >= 1 && z <= nf - 2;
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            const int ly = w + 4 * m, gy = fy0 + ly;
            const bool inn = zin && coli && gy >= 1 && gy <= nf - 2 && lres && ly >= 1 && ly <= 2 * CY + 1;
            dst[m] = inn ? f[(size_t)z * pl + (size_t)gy * nf + gx] : T(0);
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
                    fc[((size_t)Kz * nc + Y) * nc + X] = fw3<T>(Rr[sb], Rr[sc], Rr[s1], 2 * (Y - Y0) + 2,
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
// Prolongation + correction u += P uc on inner fine nodes (used when no
// post-smoothing sweep can absorb it), coarsest solve, copies.
// ---------------------------------------------------------------------------

template <typename T, int DIM>
__global__ __launch_bounds__(NT) void k_prolong(const GridDesc* __restrict__ descs, int sel) {
    const GridDesc d = descs[blockIdx.y];
    if (d.done && *d.done) return;
    const int n = d.n, nc = (n - 1) / 2 + 1, m = n - 2;
    const size_t total = DIM == 2 ? (size_t)m * m : (size_t)m * m * m;
    T* __restrict__ u = (T*)(sel ? d.t : d.u);
    const T* __restrict__ ec = (const T*)d.uc;
    for (size_t q = (size_t)blockIdx.x * NT + threadIdx.x; q < total; q += (size_t)gridDim.x * NT) {
        const int i = 1 + (int)(q % m);
        const size_t r = q / m;
        const int j = 1 + (int)(r % m);
        const int k = DIM == 2 ? 0 : 1 + (int)(r / m);
        const size_t p = ((size_t)k * n + j) * n + i;
        u[p] = u[p] + (DIM == 2 ? interp2(ec, nc, i, j) : interp3(ec, nc, i, j, k));
    }
}

// n = 3: one unknown, u = f / diag (diag = c*2d, or c*dsum).
template <typename T, int DIM, bool VAR>
__global__ void k_coarsest(const GridDesc* __restrict__ descs) {
    const GridDesc d = descs[blockIdx.x];
    if (threadIdx.x != 0 || (d.done && *d.done)) return;
    const int p = DIM == 2 ? 4 : 13;
    T* u = (T*)d.u;
    const T* f = (const T*)d.f;
    const T c = (T)d.c;
    T diag;
    if constexpr (VAR) {
        const T* k = (const T*)d.k;
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
    u[p] = f[p] / diag;
}

template <typename T>
__global__ __launch_bounds__(NT) void k_copy_t_to_u(const GridDesc* __restrict__ descs, size_t total) {
    const GridDesc d = descs[blockIdx.y];
    if (d.done && *d.done) return;
    T* __restrict__ u = (T*)d.u;
    const T* __restrict__ t = (const T*)d.t;
    for (size_t q = (size_t)blockIdx.x * NT + threadIdx.x; q < total; q += (size_t)gridDim.x * NT) u[q] = t[q];
}

template <typename T>
__global__ __launch_bounds__(NT) void k_zero_u(const GridDesc* __restrict__ descs, size_t total) {
    const GridDesc d = descs[blockIdx.y];
    if (d.done && *d.done) return;
    T* __restrict__ u = (T*)d.u;
    for (size_t q = (size_t)blockIdx.x * NT + threadIdx.x; q < total; q += (size_t)gridDim.x * NT) u[q] = T(0);
}

__global__ __launch_bounds__(NT) void k_copy_bytes(uint4* __restrict__ dst, const uint4* __restrict__ src,
                                                   size_t n16) {
    for (size_t q = (size_t)blockIdx.x * NT + threadIdx.x; q < n16; q += (size_t)gridDim.x * NT) dst[q] = src[q];
}

// ---------------------------------------------------------------------------
// FP64 residual norm partials (solve loop of the Layer-4 Application function)
// ---------------------------------------------------------------------------

template <bool VAR, int BY>
__global__ __launch_bounds__(NT) void k_norm2d(const GridDesc* __restrict__ descs, int sel, double* __restrict__ part,
                                               int pstride) {
    const GridDesc d = descs[blockIdx.y];
    __shared__ double red4[4];
    if (d.done && *d.done) return;
    constexpr int TX = BX - 2, TY = BY - 2, RPT = BY / 4;
    const int n = d.n;
    const int ntx = (n - 2 + TX - 1) / TX;
    const int tile = blockIdx.x;
    const int x0 = 1 + (tile % ntx) * TX, y0 = 1 + (tile / ntx) * TY;
    const double* __restrict__ u = (const double*)(sel ? d.t : d.u);
    const double* __restrict__ f = (const double*)d.f;
    const double* __restrict__ kf = (const double*)d.k;
    const double c = d.c;
    __shared__ double U[BY][BX];
    __shared__ double K[VAR ? BY : 1][BX];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int gx = x0 - 1 + lane;
    double fr[RPT];
#pragma unroll
    for (int m = 0; m < RPT; ++m) {
        const int ly = w + 4 * m, gy = y0 - 1 + ly;
        const bool ing = gx < n && gy < n;
        const size_t p = (size_t)gy * n + gx;
        U[ly][lane] = ing ? u[p] : 0.0;
        if constexpr (VAR) K[ly][lane] = ing ? kf[p] : 1.0;
        fr[m] = ing ? f[p] : 0.0;
    }
    __syncthreads();
    double acc = 0.0;
#pragma unroll
    for (int m = 0; m < RPT; ++m) {
        const int ly = w + 4 * m, gy = y0 - 1 + ly;
        if (lane >= 1 && lane <= BX - 2 && ly >= 1 && ly <= BY - 2 && gx <= n - 2 && gy <= n - 2) {
            double ds;
            const double r = lds_res2<double, VAR>(U, K, ly, lane, fr[m], c, ds);
            acc += r * r;
        }
    }
    const double s = block_sum(acc, red4);
    if (threadIdx.x == 0) part[(size_t)d.inst * pstride + blockIdx.x] = s;
}

template <bool VAR, int BY>
__global__ __launch_bounds__(NT) void k_norm3d(const GridDesc* __restrict__ descs, int sel, double* __restrict__ part,
                                               int pstride, int zchunk) {
    const GridDesc d = descs[blockIdx.y];
    __shared__ double red4[4];
    if (d.done && *d.done) return;
    constexpr int TX = BX - 2, TY = BY - 2, RPT = BY / 4;
    const int n = d.n;
    const int ntx = (n - 2 + TX - 1) / TX, nty = (n - 2 + TY - 1) / TY;
    const int tile = blockIdx.x;
    const int tx = tile % ntx, t2 = tile / ntx, ty = t2 % nty, tz = t2 / nty;
    const int x0 = 1 + tx * TX, y0 = 1 + ty * TY, z0 = 1 + tz * zchunk, z1 = min(z0 + zchunk, n - 1);
    const double* __restrict__ u = (const double*)(sel ? d.t : d.u);
    const double* __restrict__ f = (const double*)d.f;
    const double* __restrict__ kf = (const double*)d.k;
    const double c = d.c;
    __shared__ double U[3][BY][BX];
    __shared__ double K[VAR ? 3 : 1][BY][BX];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int gx = x0 - 1 + lane;
    const size_t pl = (size_t)n * n;
    double un[RPT], kn[RPT], fn[RPT], fc[RPT] = {};
    auto issue = [&](int z) {
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            const int gy = y0 - 1 + w + 4 * m;
            const bool ing = gx < n && gy < n && z < n;
            const size_t p = (size_t)z * pl + (size_t)gy * n + gx;
            un[m] = ing ? u[p] : 0.0;
            if constexpr (VAR) kn[m] = ing ? kf[p] : 1.0;
            fn[m] = ing ? f[p] : 0.0;
        }
    };
    double acc = 0.0;
    const int kstart = z0 - 1, kend = z1;
    issue(kstart);
    for (int kk = kstart; kk <= kend; ++kk) {
        const int s0 = (kk - kstart) % 3, s1 = (kk - 1 - kstart + 3) % 3, s2 = (kk - 2 - kstart + 6) % 3;
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            U[s0][w + 4 * m][lane] = un[m];
            if constexpr (VAR) K[s0][w + 4 * m][lane] = kn[m];
        }
        double fprev[RPT];
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            fprev[m] = fc[m];
            fc[m] = fn[m];
        }
        if (kk + 1 <= kend) issue(kk + 1);
        __syncthreads();
        const int zz = kk - 1;
        if (zz >= z0) {
#pragma unroll
            for (int m = 0; m < RPT; ++m) {
                const int ly = w + 4 * m, gy = y0 - 1 + ly;
                if (lane >= 1 && lane <= BX - 2 && ly >= 1 && ly <= BY - 2 && gx <= n - 2 && gy <= n - 2) {
                    double ds;
                    const double r =
                        lds_res3<double, VAR>(U[s2], U[s1], U[s0], K[s2], K[s1], K[s0], ly, lane, fprev[m], c, ds);
                    acc += r * r;
                }
            }
        }
        __syncthreads();
    }
    const double s = block_sum(acc, red4);
    if (threadIdx.x == 0) part[(size_t)d.inst * pstride + blockIdx.x] = s;
}

// ---------------------------------------------------------------------------
// FP64 refinement pass: u_out = u_in + e (inner), r = f - A u_out (FP64),
// r32 = (float) r on inner nodes, partial sums of r^2.
// ---------------------------------------------------------------------------

template <bool VAR, int BY>
__global__ __launch_bounds__(NT) void k_ir2d(const IRDesc* __restrict__ descs, int sel, int flags,
                                             double* __restrict__ part, int pstride) {
    const IRDesc d = descs[blockIdx.y];
    __shared__ double red4[4];
    if (d.done && *d.done) return;
    constexpr int TX = BX - 2, TY = BY - 2, RPT = BY / 4;
    const int n = d.n;
    const int ntx = (n - 2 + TX - 1) / TX;
    const int tile = blockIdx.x;
    const int x0 = 1 + (tile % ntx) * TX, y0 = 1 + (tile / ntx) * TY;
    const double* __restrict__ uin = d.u[sel];
    double* __restrict__ uout = d.u[sel ^ 1];
    const float* __restrict__ e = d.e;
    const double* __restrict__ f = d.f;
    const double* __restrict__ kf = d.k;
    float* __restrict__ r32 = d.r;
    const double c = d.c;
    __shared__ double U[BY][BX];
    __shared__ double K[VAR ? BY : 1][BX];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int gx = x0 - 1 + lane;
    double fr[RPT];
#pragma unroll
    for (int m = 0; m < RPT; ++m) {
        const int ly = w + 4 * m, gy = y0 - 1 + ly;
        const bool ing = gx < n && gy < n;
        const bool inn = gx >= 1 && gx <= n - 2 && gy >= 1 && gy <= n - 2;
        const size_t p = (size_t)gy * n + gx;
        double v = ing ? uin[p] : 0.0;
        if (inn && !(flags & IR_NO_UPDATE)) v = v + (double)e[p];
        U[ly][lane] = v;
        if constexpr (VAR) K[ly][lane] = ing ? kf[p] : 1.0;
        fr[m] = ing ? f[p] : 0.0;
    }
    __syncthreads();
    double acc = 0.0;
#pragma unroll
    for (int m = 0; m < RPT; ++m) {
        const int ly = w + 4 * m, gy = y0 - 1 + ly;
        if (lane >= 1 && lane <= BX - 2 && ly >= 1 && ly <= BY - 2 && gx <= n - 2 && gy <= n - 2) {
            const size_t p = (size_t)gy * n + gx;
            double ds;
            const double r = lds_res2<double, VAR>(U, K, ly, lane, fr[m], c, ds);
            if (!(flags & IR_NO_UPDATE)) uout[p] = U[ly][lane];
            r32[p] = (float)r;
            acc += r * r;
        }
    }
    const double s = block_sum(acc, red4);
    if (threadIdx.x == 0) part[(size_t)d.inst * pstride + blockIdx.x] = s;
}

template <bool VAR, int BY>
__global__ __launch_bounds__(NT) void k_ir3d(const IRDesc* __restrict__ descs, int sel, int flags,
                                             double* __restrict__ part, int pstride, int zchunk) {
    const IRDesc d = descs[blockIdx.y];
    __shared__ double red4[4];
    if (d.done && *d.done) return;
    constexpr int TX = BX - 2, TY = BY - 2, RPT = BY / 4;
    const int n = d.n;
    const int ntx = (n - 2 + TX - 1) / TX, nty = (n - 2 + TY - 1) / TY;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int tx = tile % ntx, t2 = tile / ntx, ty = t2 % nty, tz = t2 / nty;
    const int x0 = 1 + tx * TX, y0 = 1 + ty * TY, z0 = 1 + tz * zchunk, z1 = min(z0 + zchunk, n - 1);
    const double* __restrict__ uin = d.u[sel];
    double* __restrict__ uout = d.u[sel ^ 1];
    const float* __restrict__ e = d.e;
    const double* __restrict__ f = d.f;
    const double* __restrict__ kf = d.k;
    float* __restrict__ r32 = d.r;
    const double c = d.c;
    __shared__ double U[3][BY][BX];
    __shared__ double K[VAR ? 3 : 1][BY][BX];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int gx = x0 - 1 + lane;
    const bool coli = gx >= 1 && gx <= n - 2;
    const size_t pl = (size_t)n * n;
    double un[RPT], kn[RPT], fn[RPT], fc[RPT] = {};
    float en[RPT];
    auto issue = [&](int z) {
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            const int gy = y0 - 1 + w + 4 * m;
            const bool ing = gx < n && gy < n && z < n;
            const bool inn = coli && gy >= 1 && gy <= n - 2 && z >= 1 && z <= n - 2;
            const size_t p = (size_t)z * pl + (size_t)gy * n + gx;
            un[m] = ing ? uin[p] : 0.0;
            en[m] = (inn && !(flags & IR_NO_UPDATE)) ? e[p] : 0.0f;
            if constexpr (VAR) kn[m] = ing ? kf[p] : 1.0;
            fn[m] = inn ? f[p] : 0.0;
        }
    };
    double acc = 0.0;
    const int kstart = z0 - 1, kend = z1;
    issue(kstart);
    for (int kk = kstart; kk <= kend; ++kk) {
        const int s0 = (kk - kstart) % 3, s1 = (kk - 1 - kstart + 3) % 3, s2 = (kk - 2 - kstart + 6) % 3;
        const bool zin = kk >= 1 && kk <= n - 2;
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            const int ly = w + 4 * m, gy = y0 - 1 + ly;
            const bool inn = zin && coli && gy >= 1 && gy <= n - 2;
            const double v = inn ? un[m] + (double)en[m] : un[m];
            U[s0][ly][lane] = v;
            if constexpr (VAR) K[s0][ly][lane] = kn[m];
            // the owned part of plane kk goes to the output iterate
            if (!(flags & IR_NO_UPDATE) && inn && kk >= z0 && kk < z1 && lane >= 1 && lane <= BX - 2 && ly >= 1 &&
                ly <= BY - 2)
                uout[(size_t)kk * pl + (size_t)gy * n + gx] = v;
        }
        double fprev[RPT];
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            fprev[m] = fc[m];
            fc[m] = fn[m];
        }
        if (kk + 1 <= kend) issue(kk + 1);
        __syncthreads();
        const int zz = kk - 1;
        if (zz >= z0) {
#pragma unroll
            for (int m = 0; m < RPT; ++m) {
                const int ly = w + 4 * m, gy = y0 - 1 + ly;
                if (lane >= 1 && lane <= BX - 2 && ly >= 1 && ly <= BY - 2 && gx <= n - 2 && gy <= n - 2) {
                    double ds;
                    const double r =
                        lds_res3<double, VAR>(U[s2], U[s1], U[s0], K[s2], K[s1], K[s0], ly, lane, fprev[m], c, ds);
                    r32[(size_t)zz * pl + (size_t)gy * n + gx] = (float)r;
                    acc += r * r;
                }
            }
        }
        __syncthreads();
    }
    const double s = block_sum(acc, red4);
    if (threadIdx.x == 0) part[(size_t)d.inst * pstride + blockIdx.x] = s;
}

__global__ __launch_bounds__(NT) void k_norm_finalize(const double* __restrict__ part, int pstride, int nparts,
                                                      int row0, double* __restrict__ norm) {
    __shared__ double red4[4];
    const int row = row0 + blockIdx.x;
    const double* p = part + (size_t)row * pstride;
    double s = 0.0;
    for (int i = threadIdx.x; i < nparts; i += NT) s += p[i];
    const double t = block_sum(s, red4);
    if (threadIdx.x == 0) norm[row] = sqrt(t);
}

// Start of a solve: norm0 = norm, hist[0] = norm, steps = 0, and a zero
// initial residual is already converged.
__global__ void k_solve_init(const double* __restrict__ norm, double* __restrict__ norm0, int* __restrict__ done,
                             int* __restrict__ steps, int* __restrict__ status, double* __restrict__ hist,
                             int hstride, int ninst) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ninst) return;
    const double r = norm[i];
    norm0[i] = r;
    steps[i] = 0;
    if (hist) hist[(size_t)i * hstride] = r;
    const bool zero = r == 0.0;
    const bool bad = !(r == r) || r > 1e300;
    status[i] = bad ? -5 : (zero ? 0 : 1);
    done[i] = (zero || bad) ? 1 : 0;
}

// After each cycle: count it, record the residual, and stop the instance
// when converged (rho <= tol rho0), diverged (NaN/Inf or growth > 1e6) or
// out of cycles.  status: 1 running, 0 converged, 2 not converged, -5 diverged.
__global__ void k_stop_test(const double* __restrict__ norm, const double* __restrict__ norm0, int* __restrict__ done,
                            int* __restrict__ steps, int* __restrict__ status, double* __restrict__ hist, int hstride,
                            double tol, int max_steps, int ninst) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ninst || done[i]) return;
    const double r = norm[i], r0 = norm0[i];
    const int s = steps[i] + 1;
    steps[i] = s;
    if (hist && s < hstride) hist[(size_t)i * hstride + s] = r;
    int st = 1;
    if (!(r == r) || r > 1e300) st = -5;
    else if (r > 1e6 * r0) st = -5;
    else if (r <= tol * r0) st = 0;
    else if (s >= max_steps) st = 2;
    if (st != 1) {
        status[i] = st;
        done[i] = 1;
    }
}

// Setup helpers: coarse coefficient by injection, precision conversion, fills.
template <typename TS, typename TD>
__global__ __launch_bounds__(NT) void k_inject(const TS* __restrict__ src, int nf, TD* __restrict__ dst, int nc,
                                               int dim) {
    const size_t total = dim == 2 ? (size_t)nc * nc : (size_t)nc * nc * nc;
    for (size_t q = (size_t)blockIdx.x * NT + threadIdx.x; q < total; q += (size_t)gridDim.x * NT) {
        const int I = (int)(q % nc);
        const size_t r = q / nc;
        const int J = (int)(r % nc);
        const int K = dim == 2 ? 0 : (int)(r / nc);
        dst[q] = (TD)src[((size_t)(2 * K) * nf + 2 * J) * nf + 2 * I];
    }
}

template <typename TS, typename TD>
__global__ __launch_bounds__(NT) void k_convert(const TS* __restrict__ src, TD* __restrict__ dst, size_t total) {
    for (size_t q = (size_t)blockIdx.x * NT + threadIdx.x; q < total; q += (size_t)gridDim.x * NT) dst[q] = (TD)src[q];
}

__global__ void k_fill_int(int* __restrict__ p, int v, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

// ---------------------------------------------------------------------------
// Launch helpers
// ---------------------------------------------------------------------------

inline int cdiv(int a, int b) { return (a + b - 1) / b; }

int nzchunks(int m, int zchunk) { return cdiv(m, zchunk); }

}  // namespace

int smooth_tiles(int dim, int sm, int n, TileCfg cfg) {
    const int H = sm == SM_RBGS ? 2 : 1;
    const int TX = BX - 2 * H, TY = cfg.by - 2 * H;
    const int m = n - 2;
    if (dim == 2) return cdiv(m, TX) * cdiv(m, TY);
    return cdiv(m, TX) * cdiv(m, TY) * nzchunks(m, cfg.zchunk);
}

int restrict_tiles(int dim, int nf, TileCfg cfg) {
    const int CX = (BX - 3) / 2, CY = (cfg.by - 3) / 2;
    const int mc = (nf - 1) / 2 + 1 - 2;
    if (dim == 2) return cdiv(mc, CX) * cdiv(mc, CY);
    return cdiv(mc, CX) * cdiv(mc, CY) * nzchunks(mc, cfg.zchunk);
}

int norm_tiles(int dim, int n, TileCfg cfg) {
    const int TX = BX - 2, TY = cfg.by - 2, m = n - 2;
    if (dim == 2) return cdiv(m, TX) * cdiv(m, TY);
    return cdiv(m, TX) * cdiv(m, TY) * nzchunks(m, cfg.zchunk);
}

#define MG_BY_SWITCH(by, CALL) \
    switch (by) {              \
        case 8: {              \
            constexpr int BY = 8; \
            CALL;              \
        } break;               \
        case 16: {             \
            constexpr int BY = 16; \
            CALL;              \
        } break;               \
        case 32: {             \
            constexpr int BY = 32; \
            CALL;              \
        } break;               \
        default:               \
            return hipErrorInvalidValue; \
    }

template <typename T>
hipError_t launch_smooth(int dim, int sm, bool var, const GridDesc* d, int ninst, int n, int sel, int flags,
                         TileCfg cfg, hipStream_t s) {
    if (n < 5 || ninst <= 0) return hipErrorInvalidValue;
    const dim3 grid(smooth_tiles(dim, sm, n, cfg), ninst);
#define MG_SM(SMV, VARV)                                                                                \
    do {                                                                                                \
        if (dim == 2) {                                                                                 \
            MG_BY_SWITCH(cfg.by, (k_smooth2d<T, SMV, VARV, BY><<<grid, NT, 0, s>>>(d, sel, flags)))     \
        } else {                                                                                        \
            MG_BY_SWITCH(cfg.by, (k_smooth3d<T, SMV, VARV, BY><<<grid, NT, 0, s>>>(d, sel, flags, cfg.zchunk))) \
        }                                                                                               \
    } while (0)
    if (sm == SM_RBGS) {
        if (var) MG_SM(SM_RBGS, true);
        else MG_SM(SM_RBGS, false);
    } else {
        if (var) MG_SM(SM_JACOBI, true);
        else MG_SM(SM_JACOBI, false);
    }
#undef MG_SM
    return hipGetLastError();
}

template <typename T>
hipError_t launch_restrict(int dim, bool var, const GridDesc* d, int ninst, int nf, int sel, TileCfg cfg,
                           hipStream_t s) {
    if (nf < 5 || ninst <= 0) return hipErrorInvalidValue;
    const dim3 grid(restrict_tiles(dim, nf, cfg), ninst);
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
    const size_t m = (size_t)(nf - 2);
    const size_t total = dim == 2 ? m * m : m * m * m;
    const int blocks = (int)std::min<size_t>((total + NT - 1) / NT, 4096);
    const dim3 grid(blocks, ninst);
    if (dim == 2) k_prolong<T, 2><<<grid, NT, 0, s>>>(d, sel);
    else k_prolong<T, 3><<<grid, NT, 0, s>>>(d, sel);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_coarsest(int dim, bool var, const GridDesc* d, int ninst, hipStream_t s) {
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

hipError_t launch_norm(int dim, bool var, const GridDesc* d, int ninst, int n, int sel, double* partial, int pstride,
                       TileCfg cfg, hipStream_t s) {
    const dim3 grid(norm_tiles(dim, n, cfg), ninst);
    if ((int)grid.x > pstride) return hipErrorInvalidValue;
    if (dim == 2) {
        if (var) {
            MG_BY_SWITCH(cfg.by, (k_norm2d<true, BY><<<grid, NT, 0, s>>>(d, sel, partial, pstride)))
        } else {
            MG_BY_SWITCH(cfg.by, (k_norm2d<false, BY><<<grid, NT, 0, s>>>(d, sel, partial, pstride)))
        }
    } else {
        if (var) {
            MG_BY_SWITCH(cfg.by, (k_norm3d<true, BY><<<grid, NT, 0, s>>>(d, sel, partial, pstride, cfg.zchunk)))
        } else {
            MG_BY_SWITCH(cfg.by, (k_norm3d<false, BY><<<grid, NT, 0, s>>>(d, sel, partial, pstride, cfg.zchunk)))
        }
    }
    return hipGetLastError();
}

hipError_t launch_ir_update(int dim, bool var, const IRDesc* d, int ninst, int n, int sel, int flags,
                            double* partial, int pstride, TileCfg cfg, hipStream_t s) {
    const dim3 grid(norm_tiles(dim, n, cfg), ninst);
    if ((int)grid.x > pstride) return hipErrorInvalidValue;
    if (dim == 2) {
        if (var) {
            MG_BY_SWITCH(cfg.by, (k_ir2d<true, BY><<<grid, NT, 0, s>>>(d, sel, flags, partial, pstride)))
        } else {
            MG_BY_SWITCH(cfg.by, (k_ir2d<false, BY><<<grid, NT, 0, s>>>(d, sel, flags, partial, pstride)))
        }
    } else {
        if (var) {
            MG_BY_SWITCH(cfg.by, (k_ir3d<true, BY><<<grid, NT, 0, s>>>(d, sel, flags, partial, pstride, cfg.zchunk)))
        } else {
            MG_BY_SWITCH(cfg.by, (k_ir3d<false, BY><<<grid, NT, 0, s>>>(d, sel, flags, partial, pstride, cfg.zchunk)))
        }
    }
    return hipGetLastError();
}

hipError_t launch_norm_finalize(const double* partial, int pstride, int nparts, int row0, int ninst, double* norm,
                                hipStream_t s) {
    k_norm_finalize<<<ninst, NT, 0, s>>>(partial, pstride, nparts, row0, norm);
    return hipGetLastError();
}

hipError_t launch_solve_init(const double* norm, double* norm0, int* done, int* steps, int* status, double* hist,
                             int hstride, int ninst, hipStream_t s) {
    k_solve_init<<<cdiv(ninst, 256), 256, 0, s>>>(norm, norm0, done, steps, status, hist, hstride, ninst);
    return hipGetLastError();
}

hipError_t launch_stop_test(const double* norm, const double* norm0, int* done, int* steps, int* status, double* hist,
                            int hstride, double tol, int max_steps, int ninst, hipStream_t s) {
    k_stop_test<<<cdiv(ninst, 256), 256, 0, s>>>(norm, norm0, done, steps, status, hist, hstride, tol, max_steps,
                                                  ninst);
    return hipGetLastError();
}

template <typename TS, typename TD>
hipError_t launch_inject(int dim, int nf, const TS* src, int nc, TD* dst, hipStream_t s) {
    const size_t total = dim == 2 ? (size_t)nc * nc : (size_t)nc * nc * nc;
    const int blocks = (int)std::min<size_t>((total + NT - 1) / NT, 8192);
    k_inject<TS, TD><<<blocks, NT, 0, s>>>(src, nf, dst, nc, dim);
    return hipGetLastError();
}
template hipError_t launch_inject<double, double>(int, int, const double*, int, double*, hipStream_t);
template hipError_t launch_inject<double, float>(int, int, const double*, int, float*, hipStream_t);
template hipError_t launch_inject<float, float>(int, int, const float*, int, float*, hipStream_t);

template <typename TS, typename TD>
hipError_t launch_convert(size_t total, const TS* src, TD* dst, hipStream_t s) {
    const int blocks = (int)std::min<size_t>((total + NT - 1) / NT, 8192);
    k_convert<TS, TD><<<blocks, NT, 0, s>>>(src, dst, total);
    return hipGetLastError();
}
template hipError_t launch_convert<double, float>(size_t, const double*, float*, hipStream_t);
template hipError_t launch_convert<double, double>(size_t, const double*, double*, hipStream_t);
template hipError_t launch_convert<float, float>(size_t, const float*, float*, hipStream_t);

hipError_t launch_fill_int(int* p, int v, int count, hipStream_t s) {
    k_fill_int<<<cdiv(count, 256), 256, 0, s>>>(p, v, count);
    return hipGetLastError();
}

hipError_t launch_copy_bytes(void* dst, const void* src, size_t bytes, hipStream_t s) {
    if (bytes % 16 != 0) return hipErrorInvalidValue;
    const size_t n16 = bytes / 16;
    const int blocks = (int)std::min<size_t>((n16 + NT - 1) / NT, 8192);
    k_copy_bytes<<<blocks, NT, 0, s>>>((uint4*)dst, (const uint4*)src, n16);
    return hipGetLastError();
}

#define MG_INST(T)                                                                                              \
    template hipError_t launch_smooth<T>(int, int, bool, const GridDesc*, int, int, int, int, TileCfg,           \
                                         hipStream_t);                                                          \
    template hipError_t launch_restrict<T>(int, bool, const GridDesc*, int, int, int, TileCfg, hipStream_t);    \
    template hipError_t launch_prolong<T>(int, const GridDesc*, int, int, int, hipStream_t);                    \
    template hipError_t launch_coarsest<T>(int, bool, const GridDesc*, int, hipStream_t);                       \
    template hipError_t launch_copy_t_to_u<T>(int, const GridDesc*, int, int, hipStream_t);                     \
    template hipError_t launch_zero_u<T>(int, const GridDesc*, int, int, hipStream_t);
MG_INST(double)
MG_INST(float)

}  // namespace mg
