// 3D smoothing sweep with one wavefront per tile and the tile's rows in
// registers (included by mg_smooth3d.inl).
#pragma once

namespace mg {
namespace {

// ---------------------------------------------------------------------------
// A single wavefront marches a 64 x BY tile along z.  Lane = x position; the
// thread holds all BY rows of its column for the recent planes, so the y-
// neighbours of a node are the thread's own registers, x-neighbours come from
// the adjacent lanes (DPP) and z-neighbours from the plane rings: no LDS and
// no barriers.  Step kk (plane kk enters): red relaxation of plane kk-1 on the
// tile + one-node ring, black relaxation of plane kk-2 on the tile, written
// out.  The old values of plane kk-2 that the red relaxation needs below are
// read from the red-updated ring: a red node's z-neighbours are black, and
// black nodes keep their old values in the red half-sweep.
// ---------------------------------------------------------------------------

template <typename ST, int SM, bool VAR, int BY, int PD, int FL>
struct SweepRC {
    using T = arith_t<ST>;  // arithmetic type; ST is the storage type of u, f and the coarse correction
    static_assert(!VAR || sizeof(ST) == sizeof(T), "coefficient fields are stored in the arithmetic type");
    static constexpr int flags = FL;
    static constexpr int H = SM == SM_RBGS ? 2 : 1;
    static constexpr int TX = BX - 2 * H, TY = BY - 2 * H;
    static constexpr bool PRO = (FL & SWEEP_PROLONG) != 0;

    const MG_GLOBAL ST* __restrict__ uin;
    MG_GLOBAL ST* __restrict__ uout;
    const MG_GLOBAL ST* __restrict__ f;
    const MG_GLOBAL T* __restrict__ kf;
    const MG_GLOBAL ST* __restrict__ ec;
    int n, nc, x0, y0, z0, z1, kstart, kend;
    T c, wd, om;
    int lane, gx;
    int cfirst;  // colour relaxed in the first half-sweep (0 red, 1 black)
    bool coli, lane1, lanet;
    unsigned xb, cxb;
    size_t pl;

    T un[3][BY], kn[3][BY];  // prefetched raw u (and k)
    T uo[3][BY];             // old u of planes kk, kk-1 (and kk-2 for Jacobi)
    T ko[3][BY];             // k of planes kk, kk-1, kk-2
    T ro[3][BY];             // red-updated u of planes kk-1, kk-2, kk-3
    T fr[3][BY];             // f of planes kk, kk-1, kk-2
    T kbelow[BY];            // k of plane kk-3 (coefficient field only)
    T craw[PRO ? BY : 1][2];
    T sylast[PRO ? BY : 1];

    __device__ __forceinline__ int gy(int m) const { return y0 - H + m; }  // wave-uniform
    __device__ __forceinline__ int rowoff(int m) const { return min(max(gy(m), 0), n - 1) * n; }
    __device__ __forceinline__ bool yin(int m) const { return gy(m) >= 1 && gy(m) <= n - 2; }

    __device__ __forceinline__ void init() {
        pl = (size_t)n * n;
        const int xc = min(max(gx, 0), n - 1);
        xb = (unsigned)xc * (unsigned)sizeof(ST);
        coli = gx >= 1 && gx <= n - 2;
        lane1 = lane >= 1 && lane <= BX - 2;
        lanet = lane >= 2 && lane <= BX - 3;
        if constexpr (PRO) cxb = (unsigned)(H == 2 ? xc >> 1 : (xc + 1) >> 1) * (unsigned)sizeof(ST);
    }

    // Loads are unconditional from clamped (always in-bounds) addresses and
    // kept as loaded: only inner nodes consume them.
    __device__ __forceinline__ void issue_u(int z, T (&du)[BY], T (&dk)[BY]) {
        const size_t zoff = (size_t)min(max(z, 0), n - 1) * pl;
#pragma unroll
        for (int m = 0; m < BY; ++m) {
            if constexpr (!(flags & SWEEP_ZERO_GUESS)) du[m] = ld_off(uin + zoff + rowoff(m), xb);
            else du[m] = T(0);
            if constexpr (VAR) dk[m] = ld_off(kf + zoff + rowoff(m), xb);
        }
    }
    // f is read on the rows that are relaxed (not the outermost halo rows).
    __device__ __forceinline__ void issue_f(int z, T (&dst)[BY]) {
        const size_t zoff = (size_t)min(max(z, 0), n - 1) * pl;
#pragma unroll
        for (int m = 1; m < BY - 1; ++m) dst[m] = ld_off(f + zoff + rowoff(m), xb);
    }

    // ---- coarse-grid correction (SWEEP_PROLONG), as in the LDS variant ----
    __device__ __forceinline__ void issue_c(int K) {
        const MG_GLOBAL ST* __restrict__ cp = ec + (size_t)min(max(K, 0), nc - 1) * ((size_t)nc * nc);
#pragma unroll
        for (int m = 0; m < BY; ++m) {
            const int yc = min(max(gy(m), 0), n - 1);
            const MG_GLOBAL ST* __restrict__ r0 = cp + (yc >> 1) * nc;
            craw[m][0] = ld_off(r0, cxb);
            craw[m][1] = ld_off(r0 + ((yc & 1) ? nc : 0), cxb);
        }
    }
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
        return (min(max(gy(m), 0), n - 1) & 1) ? sa + sb : sa;
    }
    template <int S0>
    __device__ __forceinline__ void correct_entering(int kk) {
        const bool zo = (kk & 1) != 0;
        const bool zin = kk >= 1 && kk <= n - 2;
#pragma unroll
        for (int m = 0; m < BY; ++m) {
            T sum;
            if (zo) {
                const T sn = coarse_sum(m);
                sum = sylast[m] + sn;
                sylast[m] = sn;
            } else {
                sum = sylast[m];
            }
            const int nodd = (gx & 1) + (gy(m) & 1) + (zo ? 1 : 0);
            const T corr = nodd == 0 ? sum : (nodd == 1 ? T(0.5) * sum : (nodd == 2 ? T(0.25) * sum : T(0.125) * sum));
            if (zin && coli && yin(m)) un[S0][m] = stored<ST>(un[S0][m] + corr);
        }
        if (!zo) issue_c((kk + 2) >> 1);
    }

    // Relaxation of row m of a plane: A = the plane's values (centre, x via
    // DPP, y from rows m-1 / m+1), Bv / Av = values of the planes below / above.
    __device__ __forceinline__ T relax_row(const T (&A)[BY], const T (&Bv)[BY], const T (&Av)[BY], const T (&KA)[BY],
                                           const T (&KB)[BY], const T (&KU)[BY], int m, T fv) const {
        const T uc = A[m];
        const T uw = lane_prev(uc), ue = lane_next(uc);
        T kc = T(1), kw = T(1), ke = T(1), kS = T(1), kN = T(1), kb = T(1), ka = T(1);
        if constexpr (VAR) {
            kc = KA[m];
            kw = lane_prev(kc);
            ke = lane_next(kc);
            kS = KA[m - 1];
            kN = KA[m + 1];
            kb = KB[m];
            ka = KU[m];
        }
        T ds;
        const T r = res3<T, VAR>(uc, uw, ue, A[m - 1], A[m + 1], Bv[m], Av[m], kc, kw, ke, kS, kN, kb, ka, fv, c, ds);
        return relax<T, VAR>(uc, r, ds, c, wd, om);
    }

    template <int P>
    __device__ __forceinline__ void step(int kk) {
        constexpr int S0 = P, S1 = (P + 2) % 3, S2 = (P + 1) % 3;  // slots of planes kk, kk-1, kk-2
        constexpr int SN = (P + PD) % 3;
        if constexpr (PRO) correct_entering<S0>(kk);
#pragma unroll
        for (int m = 0; m < BY; ++m) {
            uo[S0][m] = un[S0][m];
            if constexpr (VAR) ko[S0][m] = kn[S0][m];
        }
        issue_f(kk, fr[S0]);
        issue_u(kk + PD, un[SN], kn[SN]);
        if constexpr (SM == SM_RBGS) {
            const int m1 = kk - 1;  // red plane
            // the red-updated ring starts as the old values: planes below the
            // first red plane keep them (they are the z-neighbours it reads)
#pragma unroll
            for (int m = 0; m < BY; ++m) ro[S1][m] = uo[S1][m];
            if (m1 >= z0 - 1) {
                const bool zin = m1 >= 1 && m1 <= n - 2;
                const bool ok = zin && lane1 && coli;
#pragma unroll
                for (int m = 1; m < BY - 1; ++m) {
                    const T v = stored<ST>(relax_row(uo[S1], ro[S2], uo[S0], ko[S1], ko[S2], ko[S0], m, fr[S1][m]));
                    if (ok && yin(m) && ((gx + gy(m) + m1) & 1) == cfirst) ro[S1][m] = v;
                }
            }
            const int m2 = kk - 2;  // black plane (output)
            if (m2 >= z0 && m2 < z1) {
                const bool ok = lanet && coli;
                MG_GLOBAL ST* __restrict__ out = uout + (size_t)m2 * pl;
#pragma unroll
                for (int m = 2; m < BY - 2; ++m) {
                    T v = ro[S2][m];
                    const T b = relax_row(ro[S2], ro[P], ro[S1], ko[S2], kbelow, ko[S1], m, fr[S2][m]);
                    if (((gx + gy(m) + m2) & 1) != cfirst) v = b;
                    if (ok && yin(m)) st_off(out + rowoff(m), xb, (ST)v);
                }
            }
            if constexpr (VAR) {
#pragma unroll
                for (int m = 0; m < BY; ++m) kbelow[m] = ko[S2][m];
            }
        } else {
            const int m1 = kk - 1;
            if (m1 >= z0 && m1 < z1) {
                const bool ok = lane1 && coli;
                MG_GLOBAL ST* __restrict__ out = uout + (size_t)m1 * pl;
#pragma unroll
                for (int m = 1; m < BY - 1; ++m) {
                    const T v = relax_row(uo[S1], uo[S2], uo[S0], ko[S1], ko[S2], ko[S0], m, fr[S1][m]);
                    if (ok && yin(m)) st_off(out + rowoff(m), xb, (ST)v);
                }
            }
        }
    }

    __device__ __forceinline__ void run() {
        init();
        int kk = kstart;
        if constexpr (PRO) {
            issue_c((kk - (kk & 1)) >> 1);
#pragma unroll
            for (int m = 0; m < BY; ++m) sylast[m] = coarse_sum(m);
            if (kk & 1) issue_c((kk + 1) >> 1);
        }
        issue_u(kk, un[0], kn[0]);
        if constexpr (PD == 2) issue_u(kk + 1, un[1], kn[1]);
#pragma unroll
        for (int m = 0; m < BY; ++m) {
            uo[1][m] = uo[2][m] = T(0);
            ro[0][m] = ro[1][m] = ro[2][m] = T(0);
            fr[0][m] = fr[1][m] = fr[2][m] = T(0);  // halo rows keep these (f is not read there)
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

template <typename ST, int SM, bool VAR, int BY, int PD, int FL>
__global__ __launch_bounds__(64) void k_smooth3d_rc(const GridDesc* __restrict__ descs, int sel, int zchunk) {
    const GridDesc d = descs[blockIdx.y];
    if (d.done && *gp(d.done)) return;
    using S = SweepRC<ST, SM, VAR, BY, PD, FL>;
    using T = arith_t<ST>;
    S s;
    const int n = d.n;
    const int ntx = (n - 2 + S::TX - 1) / S::TX, nty = (n - 2 + S::TY - 1) / S::TY;
    const int tile = sweep_tile(sel, blockIdx.x, gridDim.x);
    const int tx = tile % ntx, t2 = tile / ntx, ty = t2 % nty, tz = t2 / nty;
    s.n = n;
    s.nc = (n - 1) / 2 + 1;
    s.x0 = 1 + tx * S::TX;
    s.y0 = 1 + ty * S::TY;
    s.z0 = 1 + tz * zchunk;
    s.z1 = min(s.z0 + zchunk, n - 1);
    s.kstart = s.z0 - S::H;
    s.kend = s.z1 - 1 + S::H;
    s.uin = gp((const ST*)((sel & 1) ? d.t : d.u));
    s.uout = gp((ST*)((sel & 1) ? d.u : d.t));
    s.f = gp((const ST*)d.f);
    s.kf = gp((const T*)d.k);
    s.ec = gp((const ST*)d.uc);
    s.c = (T)d.c;
    s.wd = (T)d.wd;
    s.om = (T)d.omega;
    s.lane = threadIdx.x;
    s.cfirst = (sel & SEL_BLACK_FIRST) ? 1 : 0;
    s.gx = s.x0 - S::H + s.lane;
    s.run();
}

}  // namespace
}  // namespace mg
