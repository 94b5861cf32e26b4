// 3D smoothing sweeps, instantiated per precision by mg_smooth3d_f64.hip / mg_smooth3d_f32.hip.
#pragma once
#include "mg_kern.h"

namespace mg {
namespace {

// ---------------------------------------------------------------------------
// 3D smoothing sweep: x-y tile, marching along z through a chunk of planes.
//
// RBGS step kk (plane kk enters):
//   A  publish old u of plane kk (prefetched PD steps earlier), prefetch
//      plane kk+PD; the plane's values stay in the thread's registers and go
//      to LDS for the y-neighbours of other threads
//   B  red relaxation of plane kk-1 on the tile + one-node ring
//   C  black relaxation of plane kk-2 on the tile, written to the output
// Jacobi step kk: A as above, B relaxes plane kk-1 on the tile.
// A thread owns one x position (its lane) and rows w, w+4, ... of the box;
// z-neighbours come from its own registers, x-neighbours from the adjacent
// lanes (DPP), y-neighbours from LDS.  Register rings are indexed by
// (plane - first plane) mod 3, resolved at compile time by unrolling three
// steps; the coefficient ring for variable coefficients works the same way.
// ---------------------------------------------------------------------------

template <typename T, int SM, bool VAR, int BY, int PD, int FL>
struct Smooth3D {
    static constexpr int flags = FL;
    static constexpr int H = SM == SM_RBGS ? 2 : 1;
    static constexpr int TX = BX - 2 * H, TY = BY - 2 * H, RPT = BY / 4;

    T (*U)[BY][BX];   // old u of recent planes (y-neighbour exchange)
    T (*R)[BY][BX];   // red-updated u of recent planes
    T (*K)[BY][BX];   // coefficient of recent planes
    const MG_GLOBAL T* __restrict__ uin;
    MG_GLOBAL T* __restrict__ uout;
    const MG_GLOBAL T* __restrict__ f;
    const MG_GLOBAL T* __restrict__ kf;
    int n, x0, y0, z0, z1, kstart, kend;
    T c, wd, om;
    int lane, w, gx;
    bool colg, coli, lane1;
    T un[3][RPT], kn[3][RPT];  // prefetched raw u (and k) of planes up to kk+PD
    T uo[3][RPT];              // old u of planes kk, kk-1, kk-2 (own positions)
    T ko[3][RPT];              // k of planes kk, kk-1, kk-2
    T ro[3][RPT];              // red-updated u of planes kk-1, kk-2, kk-3
    T fr[3][RPT];              // f of planes kk, kk-1, kk-2

    __device__ __forceinline__ int gy(int m) const { return y0 - H + w + 4 * m; }

    // Per-thread addressing, computed once: the clamped (always in-bounds)
    // offset of each of the thread's rows inside a plane, and row masks.
    // A plane is addressed by a wave-uniform base pointer, so every load and
    // store is a scalar base plus a 32-bit per-lane offset.
    unsigned roff[RPT];  // clamp(y)*n + clamp(x)
    unsigned mgrid;      // bit m: row m inside the grid (x and y)
    unsigned minner;     // bit m: row m an inner node (x and y)
    unsigned mring;      // bit m: row m in the relaxed region of the first half-sweep
    unsigned mtile;      // bit m: row m in the output tile (second half-sweep)
    size_t pl;           // n*n

    __device__ __forceinline__ void init_rows() {
        pl = (size_t)n * n;
        const int xc = min(max(gx, 0), n - 1);
        mgrid = minner = mring = mtile = 0;
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            const int y = gy(m), ly = w + 4 * m;
            roff[m] = (unsigned)(min(max(y, 0), n - 1) * n + xc);
            if (colg && y >= 0 && y < n) mgrid |= 1u << m;
            if (coli && y >= 1 && y <= n - 2) minner |= 1u << m;
            if (lane1 && ly >= 1 && ly <= BY - 2) mring |= 1u << m;
            if (lane >= 2 && lane <= BX - 3 && ly >= 2 && ly <= BY - 3 && gx <= n - 2 && y <= n - 2)
                mtile |= 1u << m;
        }
    }

    // Loads are unconditional from clamped (always in-bounds) addresses and
    // the value is selected afterwards: no branches around loads, so the
    // compiler can keep the prefetches in flight across steps.
    __device__ __forceinline__ void issue_u(int z, T (&du)[RPT], T (&dk)[RPT]) {
        const bool zok = z >= 0 && z < n && z <= kend;
        const size_t zoff = (size_t)min(max(z, 0), n - 1) * pl;
        const MG_GLOBAL T* __restrict__ up = uin + zoff;
        const MG_GLOBAL T* __restrict__ kp = kf + zoff;
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            const bool ing = zok && ((mgrid >> m) & 1u);
            if constexpr (!(flags & SWEEP_ZERO_GUESS)) {
                const T v = up[roff[m]];
                du[m] = ing ? v : T(0);
            } else {
                du[m] = T(0);
            }
            if constexpr (VAR) {
                const T kv = kp[roff[m]];
                dk[m] = ing ? kv : T(1);
            }
        }
    }
    __device__ __forceinline__ void issue_f(int z, T (&dst)[RPT]) {
        const bool zin = z >= 1 && z <= n - 2;
        const MG_GLOBAL T* __restrict__ fp = f + (size_t)min(max(z, 0), n - 1) * pl;
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            const bool inn = zin && ((minner >> m) & 1u) && ((mring >> m) & 1u);
            const T v = fp[roff[m]];
            dst[m] = inn ? v : T(0);
        }
    }

    // relaxation at row m of the thread, plane values: A (centre plane
    // array in LDS for y-neighbours), own registers for centre / below / above
    __device__ __forceinline__ T relax_at(const T (*A)[BX], T uc, T ub, T ua, T uw, T ue, int ly, T kc, T kb, T ka,
                                          T kw, T ke, int kslot, T fv) const {
        T ds;
        const T uS = A[ly - 1][lane], uN = A[ly + 1][lane];
        T kS = T(1), kN = T(1);
        if constexpr (VAR) {
            kS = K[kslot][ly - 1][lane];
            kN = K[kslot][ly + 1][lane];
        }
        const T r = res3<T, VAR>(uc, uw, ue, uS, uN, ub, ua, kc, kw, ke, kS, kN, kb, ka, fv, c, ds);
        return relax<T, VAR>(uc, r, ds, c, wd, om);
    }

    template <int P>
    __device__ __forceinline__ void step(int kk) {
        constexpr int S0 = P, S1 = (P + 2) % 3, S2 = (P + 1) % 3;  // slots of planes kk, kk-1, kk-2
        constexpr int SN = (P + PD) % 3;                           // slot of plane kk+PD
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            uo[S0][m] = un[S0][m];
            U[S0][w + 4 * m][lane] = uo[S0][m];
            if constexpr (VAR) {
                ko[S0][m] = kn[S0][m];
                K[S0][w + 4 * m][lane] = ko[S0][m];
            }
        }
        issue_f(kk, fr[S0]);
        issue_u(kk + PD, un[SN], kn[SN]);
        __syncthreads();
        if constexpr (SM == SM_RBGS) {
            const int m1 = kk - 1;  // red plane
            if (m1 >= z0 - 1) {
                const bool zin = m1 >= 1 && m1 <= n - 2;
#pragma unroll
                for (int m = 0; m < RPT; ++m) {
                    const int ly = w + 4 * m, y = gy(m);
                    const T uc = uo[S1][m];
                    const T uw = lane_prev(uc), ue = lane_next(uc);
                    T kc = T(1), kw = T(1), ke = T(1), kb = T(1), ka = T(1);
                    if constexpr (VAR) {
                        kc = ko[S1][m];
                        kw = lane_prev(kc);
                        ke = lane_next(kc);
                        kb = ko[S2][m];
                        ka = ko[S0][m];
                    }
                    T v = uc;
                    if (zin && ((mring >> m) & (minner >> m) & 1u) && ((gx + y + m1) & 1) == 0)
                        v = relax_at(U[S1], uc, uo[S2][m], uo[S0][m], uw, ue, ly, kc, kb, ka, kw, ke, S1,
                                         fr[S1][m]);
                    ro[S1][m] = v;
                    R[S1][ly][lane] = v;
                }
            }
            __syncthreads();
            const int m2 = kk - 2;  // black plane (output)
            if (m2 >= z0 && m2 < z1) {
#pragma unroll
                for (int m = 0; m < RPT; ++m) {
                    const int ly = w + 4 * m, y = gy(m);
                    const T rc = ro[S2][m];
                    const T rw = lane_prev(rc), re = lane_next(rc);
                    T kc = T(1), kw = T(1), ke = T(1), kb = T(1), ka = T(1);
                    if constexpr (VAR) {
                        // planes kk-3 .. kk-1: ko slot P now holds plane kk, so plane kk-3 comes from kbelow
                        kc = ko[S2][m];
                        kw = lane_prev(kc);
                        ke = lane_next(kc);
                        kb = kbelow[m];
                        ka = ko[S1][m];
                    }
                    if ((mtile >> m) & 1u) {
                        T v = rc;
                        if (((gx + y + m2) & 1) == 1)
                            v = relax_at(R[S2], rc, ro[P][m], ro[S1][m], rw, re, ly, kc, kb, ka, kw, ke, S2,
                                             fr[S2][m]);
                        uout[(size_t)m2 * pl + roff[m]] = v;
                    }
                }
            }
            if constexpr (VAR) {
#pragma unroll
                for (int m = 0; m < RPT; ++m) kbelow[m] = ko[S2][m];  // k of plane kk-2 = "below" next step
            }
        } else {
            const int m1 = kk - 1;
            if (m1 >= z0 && m1 < z1) {
#pragma unroll
                for (int m = 0; m < RPT; ++m) {
                    const int ly = w + 4 * m, y = gy(m);
                    const T uc = uo[S1][m];
                    const T uw = lane_prev(uc), ue = lane_next(uc);
                    T kc = T(1), kw = T(1), ke = T(1), kb = T(1), ka = T(1);
                    if constexpr (VAR) {
                        kc = ko[S1][m];
                        kw = lane_prev(kc);
                        ke = lane_next(kc);
                        kb = ko[S2][m];
                        ka = ko[S0][m];
                    }
                    if (((mring >> m) & (minner >> m) & 1u))
                        uout[(size_t)m1 * pl + roff[m]] = relax_at(U[S1], uc, uo[S2][m], uo[S0][m], uw, ue, ly, kc,
                                                                   kb, ka, kw, ke, S1, fr[S1][m]);
                }
            }
        }
        // LDS slots written next step: U and R never collide with this step's
        // reads (three-slot rings); the coefficient slot of plane kk-2 does.
        if constexpr (VAR) __syncthreads();
    }

    T kbelow[VAR ? RPT : 1];  // k of plane kk-3 for the black relaxation

    __device__ __forceinline__ void run() {
        init_rows();
        int kk = kstart;
        issue_u(kk, un[0], kn[0]);
        if constexpr (PD == 2) issue_u(kk + 1, un[1], kn[1]);
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            uo[1][m] = uo[2][m] = T(0);
            ro[0][m] = ro[1][m] = ro[2][m] = T(0);
            ko[1][m] = ko[2][m] = T(1);
            if constexpr (VAR) kbelow[m] = T(1);
        }
        for (; kk + 2 <= kend; kk += 3) {
            step<0>(kk);
            step<1>(kk + 1);
            step<2>(kk + 2);
        }
        if (kk <= kend) step<0>(kk);
        if (kk + 1 <= kend) step<1>(kk + 1);
    }
};

template <typename T, int SM, bool VAR, int BY, int PD, int FL>
__global__ __launch_bounds__(NT) void k_smooth3d(const GridDesc* __restrict__ descs, int sel, int zchunk) {
    const GridDesc d = descs[blockIdx.y];
    if (d.done && *gp(d.done)) return;
    using S = Smooth3D<T, SM, VAR, BY, PD, FL>;
    __shared__ T U[3][BY][BX];
    __shared__ T R[SM == SM_RBGS ? 3 : 1][BY][BX];
    __shared__ T K[VAR ? 3 : 1][BY][BX];
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
    s.uin = gp((const T*)(sel ? d.t : d.u));
    s.uout = gp((T*)(sel ? d.u : d.t));
    s.f = gp((const T*)d.f);
    s.kf = gp((const T*)d.k);
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

}  // namespace

template <typename T, int SMV, bool VARV, int FL>
hipError_t launch_smooth3d_fl(const GridDesc* d, int sel, TileCfg cfg, dim3 grid, hipStream_t s) {
    if (cfg.pd == 2) {
        MG_BY_SWITCH(cfg.by, (k_smooth3d<T, SMV, VARV, BY, 2, FL><<<grid, NT, 0, s>>>(d, sel, cfg.zchunk)))
    } else {
        MG_BY_SWITCH(cfg.by, (k_smooth3d<T, SMV, VARV, BY, 1, FL><<<grid, NT, 0, s>>>(d, sel, cfg.zchunk)))
    }
    return hipSuccess;
}

template <typename T>
hipError_t launch_smooth3d(int sm, bool var, const GridDesc* d, int sel, int flags, TileCfg cfg, dim3 grid,
                           hipStream_t s) {
#define MG_FL(SMV, VARV)                                                                                   \
    switch (flags) {                                                                                       \
        case 0: return launch_smooth3d_fl<T, SMV, VARV, 0>(d, sel, cfg, grid, s);                           \
        case SWEEP_ZERO_GUESS: return launch_smooth3d_fl<T, SMV, VARV, SWEEP_ZERO_GUESS>(d, sel, cfg, grid, s); \
        default: return hipErrorInvalidValue;                                                              \
    }
    if (sm == SM_RBGS) {
        if (var) MG_FL(SM_RBGS, true) else MG_FL(SM_RBGS, false)
    } else {
        if (var) MG_FL(SM_JACOBI, true) else MG_FL(SM_JACOBI, false)
    }
#undef MG_FL
}

template hipError_t launch_smooth3d<MG_T>(int, bool, const GridDesc*, int, int, TileCfg, dim3, hipStream_t);

}  // namespace mg
