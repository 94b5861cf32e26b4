// 3D smoothing sweeps, instantiated per precision by mg_smooth3d_f64.hip / mg_smooth3d_f32.hip.
#pragma once
#include "mg_kern.h"
#include "mg_smooth3d_rc.inl"
#include "mg_smooth3d_rc2.inl"

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
// (with the black-first bit of the select argument the two colours swap
// roles: the post-smoothing sweeps of the symmetric red-black smoother).
// Jacobi step kk: A as above, B relaxes plane kk-1 on the tile.
// A thread owns one x position (its lane) and rows w, w+4, ... of the box;
// z-neighbours come from its own registers, x-neighbours from the adjacent
// lanes (DPP), y-neighbours from LDS.  Register rings are indexed by
// (plane - first plane) mod 3, resolved at compile time by unrolling three
// steps.  With variable coefficients the level's face coefficients (the +x,
// +y and +z face of every node, formed once per level at setup by the same
// harmonic mean) are prefetched with u and kept in rings of their own: +x
// and +y as the plane enters (the -x face from the neighbouring lane, the -y
// face through LDS from the row below), +z one step later (the -z face is
// the +z face of the plane below), so a sweep divides nothing.
//
// With SWEEP_PROLONG the incoming iterate is u + P uc (trilinear correction
// from the coarse grid, inner nodes only), formed as each plane enters.  A
// coarse plane K serves fine planes 2K-1, 2K and 2K+1, so each coarse plane is
// loaded once per march (issued one step ahead) and reduced per thread row to
// its x-then-y partial sum; the odd-x partner value comes from the next lane.
// ---------------------------------------------------------------------------

template <typename ST, int SM, bool VAR, int BY, int PD, int FL, int WV>
struct Smooth3D {
    using T = arith_t<ST>;  // arithmetic type; ST is the storage type of u, f and the coarse correction
    static_assert(!VAR || sizeof(ST) == sizeof(T), "coefficient fields are stored in the arithmetic type");
    static constexpr int flags = FL;
    static constexpr int H = SM == SM_RBGS ? 2 : 1;
    static constexpr int TX = BX - 2 * H, TY = BY - 2 * H, RPT = BY / WV;  // WV wavefronts, RPT rows each
    static_assert(RPT >= 1 && RPT * WV == BY, "tile rows must be a multiple of the wavefronts");

    static constexpr bool PRO = (FL & SWEEP_PROLONG) != 0;
    static constexpr bool NRM = (FL & SWEEP_NORM) != 0;
    static_assert(!NRM || sizeof(T) == 8, "the sweep's norm sums FP64 residuals");

    T (*U)[BY][BX];   // old u of recent planes (y-neighbour exchange)
    T (*R)[BY][BX];   // red-updated u of recent planes
    T (*K)[BY][BX];   // +y face coefficients of recent planes (-y faces of the rows above)
    const MG_GLOBAL ST* __restrict__ uin;
    MG_GLOBAL ST* __restrict__ uout;
    const MG_GLOBAL ST* __restrict__ f;
    const MG_GLOBAL T* __restrict__ fxa;  // face coefficients: +x at fxa, +y at fxa + n^3, +z at fxa + 2 n^3
    int n, x0, y0, z0, z1, kstart, kend;
    T c, wd, om;
    int lane, w, gx;
    int cfirst;  // colour relaxed in the first half-sweep (0 red, 1 black)
    bool colg, coli, lane1;
    T un[3][RPT];              // prefetched raw u of planes up to kk+PD
    // prefetched +x, +y, +z face coefficients (VAR) of planes up to kk+PD
    T px[VAR ? 3 : 1][RPT], py[VAR ? 3 : 1][RPT], pz[VAR ? 3 : 1][RPT];
    T uo[3][RPT];              // old u of planes kk, kk-1, kk-2 (own positions)
    T ro[3][RPT];              // red-updated u of planes kk-1, kk-2, kk-3
    T fr[3][RPT];              // f of planes kk, kk-1, kk-2
    // face coefficients (VAR) of planes kk, kk-1, kk-2: +x, -y, +y faces of
    // the node, and the +z face (to the plane above; set one step after the
    // plane enters, when the +z face of the plane three below is no longer read)
    T fxc[VAR ? 3 : 1][RPT], fys[VAR ? 3 : 1][RPT], fyn[VAR ? 3 : 1][RPT], fzc[VAR ? 3 : 1][RPT];
    double nacc;  // SWEEP_NORM: this thread's sum of r^2 of the incoming iterate over its output nodes

    __device__ __forceinline__ int gy(int m) const { return y0 - H + w + WV * m; }

    // Addressing: a thread's rows are wave-uniform (the wave index is read
    // into a scalar register), so each row of a plane has a scalar base
    // address and the only per-lane part is the byte offset of the lane's
    // (clamped, always in-bounds) x position.
    unsigned xb;         // clamp(x) * sizeof(ST)
    unsigned minner;     // bit m: row m an inner node (x and y)
    unsigned mring;      // bit m: row m in the relaxed region of the first half-sweep
    unsigned mtile;      // bit m: row m in the output tile (second half-sweep)
    size_t pl;           // n*n

    __device__ __forceinline__ int rowoff(int m) const { return min(max(gy(m), 0), n - 1) * n; }

    // coarse-grid correction (SWEEP_PROLONG)
    const MG_GLOBAL ST* __restrict__ ec;  // coarse correction, edge nc
    int nc;
    unsigned codd;                       // bit m: row m has odd y
    unsigned cxb;                        // byte offset of the lane's coarse column
    T craw[PRO ? RPT : 1][2];            // coarse rows y/2 and y/2 + (y odd) of the pending coarse plane
    T sylast[PRO ? RPT : 1];             // x-y partial sum of the latest completed coarse plane

    __device__ __forceinline__ int crowoff(int m) const { return (min(max(gy(m), 0), n - 1) >> 1) * nc; }

    __device__ __forceinline__ void init_rows() {
        pl = (size_t)n * n;
        const int xc = min(max(gx, 0), n - 1);
        xb = (unsigned)xc * (unsigned)sizeof(ST);
        minner = mring = mtile = 0;
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            const int y = gy(m), ly = w + WV * m;
            if (coli && y >= 1 && y <= n - 2) minner |= 1u << m;
            if (lane1 && ly >= 1 && ly <= BY - 2) mring |= 1u << m;
            if (lane >= 2 && lane <= BX - 3 && ly >= 2 && ly <= BY - 3 && gx <= n - 2 && y <= n - 2)
                mtile |= 1u << m;
        }
        if constexpr (PRO) {
            cxb = (unsigned)(H == 2 ? xc >> 1 : (xc + 1) >> 1) * (unsigned)sizeof(ST);
            codd = 0;
#pragma unroll
            for (int m = 0; m < RPT; ++m)
                if (min(max(gy(m), 0), n - 1) & 1) codd |= 1u << m;
        }
    }

    // Coarse plane K (clamped): for each row, the coarse row y/2 and, for odd
    // y, the row above it (the same row again for even y).
    __device__ __forceinline__ void issue_c(int K) {
        const MG_GLOBAL ST* __restrict__ cp = ec + (size_t)min(max(K, 0), nc - 1) * ((size_t)nc * nc);
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            const MG_GLOBAL ST* __restrict__ row = cp + crowoff(m);
            craw[m][0] = ld_off(row, cxb);
            craw[m][1] = ld_off(row + (((codd >> m) & 1u) ? nc : 0), cxb);
        }
    }
    // x-then-y partial sum of the pending coarse plane at row m.  Each lane
    // holds one coarse column; an odd-x lane takes its other column from a
    // neighbouring lane.  With a two-node halo (RBGS) the first lane has odd x
    // and the last even x, so lanes hold column x/2 and odd lanes pair with the
    // next lane; with a one-node halo (Jacobi) it is the other way round, so
    // lanes hold column (x+1)/2 and odd lanes pair with the previous lane.
    __device__ __forceinline__ T coarse_sum(int m) const {
        const T a = craw[m][0], b = craw[m][1];
        const bool xo = (gx & 1) != 0;
        T sa, sb;
        if constexpr (H == 2) {
            const T an = lane_next(a), bn = lane_next(b);
            sa = xo ? a + an : a;
            sb = xo ? b + bn : b;
        } else {
            const T ap = lane_prev(a), bp = lane_prev(b);
            sa = xo ? ap + a : a;
            sb = xo ? bp + b : b;
        }
        return ((codd >> m) & 1u) ? sa + sb : sa;
    }
    // Plane kk enters: add the interpolated correction on inner nodes, then
    // issue the coarse plane the next (odd) fine plane needs.
    template <int S0>
    __device__ __forceinline__ void correct_entering(int kk) {
        const bool zo = (kk & 1) != 0;
        const bool zin = kk >= 1 && kk <= n - 2;
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            T sum;
            if (zo) {
                const T sn = coarse_sum(m);
                sum = sylast[m] + sn;
                sylast[m] = sn;
            } else {
                sum = sylast[m];
            }
            const int nodd = (gx & 1) + (int)((codd >> m) & 1u) + (zo ? 1 : 0);
            const T corr = nodd == 0 ? sum : (nodd == 1 ? T(0.5) * sum : (nodd == 2 ? T(0.25) * sum : T(0.125) * sum));
            if (zin && ((minner >> m) & 1u)) un[S0][m] = stored<ST>(un[S0][m] + corr);
        }
        if (!zo) issue_c((kk + 2) >> 1);
    }

    // Loads are unconditional from clamped (always in-bounds) addresses and
    // the values are kept as loaded: a value at a position outside the grid is
    // never used, because every relaxation is taken at an inner node, whose
    // neighbours all lie in the grid.  With no select on loaded values there is
    // no branch around the loads, so the prefetches stay in flight across steps.
    template <int SL>
    __device__ __forceinline__ void issue_u(int z) {
        const size_t zoff = (size_t)min(max(z, 0), n - 1) * pl;
        const MG_GLOBAL ST* __restrict__ up = uin + zoff;
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            if constexpr (!(flags & SWEEP_ZERO_GUESS)) un[SL][m] = ld_off(up + rowoff(m), xb);
            else un[SL][m] = T(0);
        }
        if constexpr (VAR) {
            const size_t N = pl * (size_t)n;
            const MG_GLOBAL T* __restrict__ xp = fxa + zoff;
#pragma unroll
            for (int m = 0; m < RPT; ++m) {
                const MG_GLOBAL T* __restrict__ row = xp + rowoff(m);
                px[SL][m] = ld_off(row, xb);
                py[SL][m] = ld_off(row + N, xb);
                pz[SL][m] = ld_off(row + 2 * N, xb);
            }
        }
    }
    // f is read on the rows that are relaxed (not the outermost halo rows).
    __device__ __forceinline__ void issue_f(int z, T (&dst)[RPT]) {
        const MG_GLOBAL ST* __restrict__ fp = f + (size_t)min(max(z, 0), n - 1) * pl;
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            const int ly = w + WV * m;  // wave-uniform
            if (ly >= 1 && ly <= BY - 2) dst[m] = ld_off(fp + rowoff(m), xb);
        }
    }

    // relaxation at row m of the thread, plane values: A (centre plane
    // array in LDS for y-neighbours), own registers for centre / below / above;
    // QC / QB: ring slots of the node's plane and of the plane below (faces);
    // kxw: the -x face, from the neighbouring lane (taken with every lane active)
    template <int QC, int QB>
    __device__ __forceinline__ T res_at(const T (*A)[BX], T uc, T ub, T ua, T uw, T ue, int ly, int m, T kxw, T fv,
                                        T& ds) const {
        const T uS = A[ly - 1][lane], uN = A[ly + 1][lane];
        if constexpr (VAR) {
            return res_var3f(uc, uw, ue, uS, uN, ub, ua, kxw, fxc[QC][m], fys[QC][m], fyn[QC][m], fzc[QB][m],
                             fzc[QC][m], fv, c, ds);
        } else {
            ds = T(0);
            return res_lap3(uc, uw, ue, uS, uN, ub, ua, fv, c);
        }
    }
    template <int QC, int QB>
    __device__ __forceinline__ T relax_at(const T (*A)[BX], T uc, T ub, T ua, T uw, T ue, int ly, int m, T kxw,
                                          T fv) const {
        T ds;
        const T r = res_at<QC, QB>(A, uc, ub, ua, uw, ue, ly, m, kxw, fv, ds);
        return relax<T, VAR>(uc, r, ds, c, wd, om);
    }

    // -y faces of the plane that entered (slot S0): the +y faces of the rows
    // below, published in K.
    template <int S0>
    __device__ __forceinline__ void faces_below() {
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            const int ly = w + WV * m;  // wave-uniform
            if (ly >= 1 && ly <= BY - 2) fys[S0][m] = K[S0][ly - 1][lane];
        }
    }

    template <int P>
    __device__ __forceinline__ void step(int kk) {
        constexpr int S0 = P, S1 = (P + 2) % 3, S2 = (P + 1) % 3;  // slots of planes kk, kk-1, kk-2
        constexpr int SN = (P + PD) % 3;                           // slot of plane kk+PD
        if constexpr (PRO) correct_entering<S0>(kk);
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            uo[S0][m] = un[S0][m];
            U[S0][w + WV * m][lane] = uo[S0][m];
            if constexpr (VAR) {
                // before this step's prefetch reuses slot S1 (PD = 2)
                fxc[S0][m] = px[S0][m];
                fyn[S0][m] = py[S0][m];
                K[S0][w + WV * m][lane] = py[S0][m];
                fzc[S1][m] = pz[S1][m];
            }
        }
        issue_f(kk, fr[S0]);
        issue_u<SN>(kk + PD);
        __syncthreads();
        if constexpr (VAR) faces_below<S0>();
        if constexpr (SM == SM_RBGS) {
            const int m1 = kk - 1;  // red plane
            if (m1 >= z0 - 1) {
                const bool zin = m1 >= 1 && m1 <= n - 2;
#pragma unroll
                for (int m = 0; m < RPT; ++m) {
                    const int ly = w + WV * m, y = gy(m);
                    const T uc = uo[S1][m];
                    const T uw = lane_prev(uc), ue = lane_next(uc);
                    const T kxw = VAR ? lane_prev(fxc[VAR ? S1 : 0][m]) : T(0);
                    T v = uc;
                    if constexpr (NRM) {
                        // the residual of every node of the relaxed region on the
                        // incoming values; summed over the output nodes
                        if (zin && ((mring >> m) & (minner >> m) & 1u)) {
                            T ds;
                            const T r = res_at<S1, S2>(U[S1], uc, uo[S2][m], uo[S0][m], uw, ue, ly, m, kxw,
                                                       fr[S1][m], ds);
                            if (((gx + y + m1) & 1) == cfirst) v = stored<ST>(relax<T, VAR>(uc, r, ds, c, wd, om));
                            if (m1 >= z0 && m1 < z1 && ((mtile >> m) & 1u)) nacc += r * r;
                        }
                    } else {
                        if (zin && ((mring >> m) & (minner >> m) & 1u) && ((gx + y + m1) & 1) == cfirst)
                            v = stored<ST>(
                                relax_at<S1, S2>(U[S1], uc, uo[S2][m], uo[S0][m], uw, ue, ly, m, kxw, fr[S1][m]));
                    }
                    ro[S1][m] = v;
                    R[S1][ly][lane] = v;
                }
            }
            __syncthreads();
            const int m2 = kk - 2;  // black plane (output)
            if (m2 >= z0 && m2 < z1) {
#pragma unroll
                for (int m = 0; m < RPT; ++m) {
                    const int ly = w + WV * m, y = gy(m);
                    const T rc = ro[S2][m];
                    const T rw = lane_prev(rc), re = lane_next(rc);
                    const T kxw = VAR ? lane_prev(fxc[VAR ? S2 : 0][m]) : T(0);
                    if ((mtile >> m) & 1u) {
                        T v = rc;
                        // faces of plane kk-2 (slot S2); +z faces of plane kk-3 in slot P
                        if (((gx + y + m2) & 1) != cfirst)
                            v = relax_at<S2, P>(R[S2], rc, ro[P][m], ro[S1][m], rw, re, ly, m, kxw, fr[S2][m]);
                        st_off(uout + (size_t)m2 * pl + rowoff(m), xb, (ST)v);
                    }
                }
            }
        } else {
            const int m1 = kk - 1;
            if (m1 >= z0 && m1 < z1) {
#pragma unroll
                for (int m = 0; m < RPT; ++m) {
                    const int ly = w + WV * m, y = gy(m);
                    const T uc = uo[S1][m];
                    const T uw = lane_prev(uc), ue = lane_next(uc);
                    const T kxw = VAR ? lane_prev(fxc[VAR ? S1 : 0][m]) : T(0);
                    if (((mring >> m) & (minner >> m) & 1u)) {
                        T ds;
                        const T r = res_at<S1, S2>(U[S1], uc, uo[S2][m], uo[S0][m], uw, ue, ly, m, kxw, fr[S1][m], ds);
                        if constexpr (NRM) nacc += r * r;
                        st_off(uout + (size_t)m1 * pl + rowoff(m), xb, (ST)relax<T, VAR>(uc, r, ds, c, wd, om));
                    }
                }
            }
        }
        // LDS slots written next step never collide with this step's reads
        // (three-slot rings; K is read only in the step its plane enters).
    }

    __device__ __forceinline__ void run() {
        init_rows();
        int kk = kstart;
        if constexpr (PRO) {
            // plane kstart needs the coarse plane kstart/2 (rounded down) completed,
            // and for odd kstart the next coarse plane pending
            issue_c((kk - (kk & 1)) >> 1);
#pragma unroll
            for (int m = 0; m < RPT; ++m) sylast[m] = coarse_sum(m);
            if (kk & 1) issue_c((kk + 1) >> 1);
        }
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            uo[1][m] = uo[2][m] = T(0);
            ro[0][m] = ro[1][m] = ro[2][m] = T(0);
            fr[0][m] = fr[1][m] = fr[2][m] = T(0);  // halo rows keep these (f is not read there)
            if constexpr (VAR) {
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    fxc[q][m] = fys[q][m] = fyn[q][m] = fzc[q][m] = T(1);
                    px[q][m] = py[q][m] = pz[q][m] = T(1);  // planes before the march: never read
                }
            }
        }
        issue_u<0>(kk);
        if constexpr (PD == 2) issue_u<1>(kk + 1);
        for (; kk + 2 <= kend; kk += 3) {
            step<0>(kk);
            step<1>(kk + 1);
            step<2>(kk + 2);
        }
        if (kk <= kend) step<0>(kk);
        if (kk + 1 <= kend) step<1>(kk + 1);
    }
};

template <typename ST, int SM, bool VAR, int BY, int PD, int FL, int WV>
__global__ __launch_bounds__(64 * WV) void k_smooth3d(const GridDesc* __restrict__ descs, int sel, int zchunk) {
    const GridDesc d = descs[blockIdx.y];
    if (d.done && *gp(d.done)) return;
    using S = Smooth3D<ST, SM, VAR, BY, PD, FL, WV>;
    using T = arith_t<ST>;
    __shared__ T U[3][BY][BX];
    __shared__ T R[SM == SM_RBGS ? 3 : 1][BY][BX];
    __shared__ T K[VAR ? 3 : 1][BY][BX];
    S s;
    s.U = U;
    s.R = R;
    s.K = K;
    const int n = d.n;
    const int ntx = (n - 2 + S::TX - 1) / S::TX, nty = (n - 2 + S::TY - 1) / S::TY;
    const int tile = sweep_tile(sel, blockIdx.x, gridDim.x);
    const int tx = tile % ntx, t2 = tile / ntx, ty = t2 % nty, tz = t2 / nty;
    s.n = n;
    s.x0 = 1 + tx * S::TX;
    s.y0 = 1 + ty * S::TY;
    s.z0 = 1 + tz * zchunk;
    s.z1 = min(s.z0 + zchunk, n - 1);
    s.kstart = s.z0 - S::H;
    s.kend = s.z1 - 1 + S::H;
    s.uin = gp((const ST*)((sel & 1) ? d.t : d.u));
    s.uout = gp((ST*)((sel & 1) ? d.u : d.t));
    s.f = gp((const ST*)d.f);
    s.fxa = gp((const T*)d.fx);
    s.ec = gp((const ST*)d.uc);
    s.nc = (n - 1) / 2 + 1;
    s.c = (T)d.c;
    s.wd = (T)d.wd;
    s.om = (T)d.omega;
    s.lane = threadIdx.x & 63;
    s.w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    s.cfirst = (sel & SEL_BLACK_FIRST) ? 1 : 0;
    s.gx = s.x0 - S::H + s.lane;
    s.colg = s.gx >= 0 && s.gx < n;
    s.coli = s.gx >= 1 && s.gx <= n - 2;
    s.lane1 = s.lane >= 1 && s.lane <= BX - 2;
    s.nacc = 0.0;
    s.run();
    if constexpr (S::NRM) {
        // per-workgroup partial in a fixed order (finalised in block order)
        __shared__ double red[WV];
        const double tot = block_sum_w<WV>(s.nacc, red);
        if (threadIdx.x == 0) gp(d.npart)[blockIdx.x] = tot;
    }
}

}  // namespace

template <typename T, int SMV, bool VARV, int FL, int BY, int WV>
hipError_t launch_smooth3d_g(const GridDesc* d, int sel, TileCfg cfg, dim3 grid, hipStream_t s) {
    const int arg = sweep_arg(sel, cfg);
    if (cfg.pd == 2) k_smooth3d<T, SMV, VARV, BY, 2, FL, WV><<<grid, 64 * WV, 0, s>>>(d, arg, cfg.zchunk);
    else k_smooth3d<T, SMV, VARV, BY, 1, FL, WV><<<grid, 64 * WV, 0, s>>>(d, arg, cfg.zchunk);
    return hipSuccess;
}

template <typename T, int SMV, bool VARV, int FL, int BY>
hipError_t launch_smooth3d_rc(const GridDesc* d, int sel, TileCfg cfg, dim3 grid, hipStream_t s) {
    const int arg = sweep_arg(sel, cfg);
    if (cfg.pd == 2) k_smooth3d_rc<T, SMV, VARV, BY, 2, FL><<<grid, 64, 0, s>>>(d, arg, cfg.zchunk);
    else k_smooth3d_rc<T, SMV, VARV, BY, 1, FL><<<grid, 64, 0, s>>>(d, arg, cfg.zchunk);
    return hipSuccess;
}

// Tile geometries (rows x wavefronts): 8x4, 16x4, 32x4 (FP32 Laplacian only:
// eight rows per thread), 16x8 and 32x8; 8x1 and 12x1 in registers.

template <typename T, int SMV, bool VARV, int FL>
hipError_t launch_smooth3d_fl(const GridDesc* d, int sel, TileCfg cfg, dim3 grid, hipStream_t s) {
    constexpr bool wide = sizeof(arith_t<T>) == 4 && !VARV;
    constexpr bool fp64var = sizeof(arith_t<T>) == 8 && VARV;  // two rows per thread at most
    if (cfg.wv == 1) {  // one wavefront per tile, rows in registers: 8 rows, or 12 in FP32 without coefficients
        if constexpr ((sizeof(arith_t<T>) == 8 && VARV) || (FL & SWEEP_NORM) != 0) {
            return hipErrorInvalidValue;
        } else {
            switch (cfg.by) {
                case 8: return launch_smooth3d_rc<T, SMV, VARV, FL, 8>(d, sel, cfg, grid, s);
                case 12:
                    if constexpr (wide) return launch_smooth3d_rc<T, SMV, VARV, FL, 12>(d, sel, cfg, grid, s);
                    return hipErrorInvalidValue;
                default: return hipErrorInvalidValue;
            }
        }
    }
    if (cfg.wv == 4) {
        switch (cfg.by) {
            case 8: return launch_smooth3d_g<T, SMV, VARV, FL, 8, 4>(d, sel, cfg, grid, s);
            case 16:
                if constexpr (!fp64var) return launch_smooth3d_g<T, SMV, VARV, FL, 16, 4>(d, sel, cfg, grid, s);
                return hipErrorInvalidValue;
            case 32:
                if constexpr (wide) return launch_smooth3d_g<T, SMV, VARV, FL, 32, 4>(d, sel, cfg, grid, s);
                return hipErrorInvalidValue;
            default: return hipErrorInvalidValue;
        }
    }
    if (cfg.wv == 8) {
        switch (cfg.by) {
            case 16: return launch_smooth3d_g<T, SMV, VARV, FL, 16, 8>(d, sel, cfg, grid, s);
            case 32:
                if constexpr (!fp64var) return launch_smooth3d_g<T, SMV, VARV, FL, 32, 8>(d, sel, cfg, grid, s);
                return hipErrorInvalidValue;
            default: return hipErrorInvalidValue;
        }
    }
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_smooth3d(int sm, bool var, const GridDesc* d, int sel, int flags, TileCfg cfg, dim3 grid,
                           hipStream_t s) {
#define MG_FL(SMV, VARV)                                                                                   \
    switch (flags) {                                                                                       \
        case 0: return launch_smooth3d_fl<T, SMV, VARV, 0>(d, sel, cfg, grid, s);                           \
        case SWEEP_ZERO_GUESS: return launch_smooth3d_fl<T, SMV, VARV, SWEEP_ZERO_GUESS>(d, sel, cfg, grid, s); \
        case SWEEP_PROLONG: return launch_smooth3d_fl<T, SMV, VARV, SWEEP_PROLONG>(d, sel, cfg, grid, s);       \
        case SWEEP_NORM:                                                                                   \
            if constexpr (sizeof(T) == 8) return launch_smooth3d_fl<T, SMV, VARV, SWEEP_NORM>(d, sel, cfg, grid, s); \
            return hipErrorInvalidValue;                                                                   \
        default: return hipErrorInvalidValue;                                                              \
    }
    if constexpr (sizeof(T) == 2) {  // binary16 storage: Laplacian only
        if (var) return hipErrorInvalidValue;
        if (sm == SM_RBGS) MG_FL(SM_RBGS, false) else MG_FL(SM_JACOBI, false)
    } else {
        if (sm == SM_RBGS) {
            if (var) MG_FL(SM_RBGS, true) else MG_FL(SM_RBGS, false)
        } else {
            if (var) MG_FL(SM_JACOBI, true) else MG_FL(SM_JACOBI, false)
        }
    }
#undef MG_FL
}

template hipError_t launch_smooth3d<MG_T>(int, bool, const GridDesc*, int, int, TileCfg, dim3, hipStream_t);

template <typename T>
hipError_t launch_smooth3d_zg2(const GridDesc* d, int ninst, int n, int sel, TileCfg cfg, hipStream_t s) {
    if constexpr (sizeof(T) == 8) {
        return hipErrorInvalidValue;  // built for FP32 and binary16 storage
    } else {
        if (n < 5 || ninst <= 0 || cfg.zchunk < 1) return hipErrorInvalidValue;
        const dim3 grid(smooth2_tiles(n, cfg), ninst);
        const int arg = sweep_arg(sel, cfg);
        switch (cfg.by) {
            case 12: k_smooth3d_zg2<T, 12><<<grid, 64, 0, s>>>(d, arg, cfg.zchunk); break;
            case 16: k_smooth3d_zg2<T, 16><<<grid, 64, 0, s>>>(d, arg, cfg.zchunk); break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
}
template hipError_t launch_smooth3d_zg2<MG_T>(const GridDesc*, int, int, int, TileCfg, hipStream_t);

}  // namespace mg
