// 2D smoothing sweeps (omega-Jacobi, fused red-black Gauss-Seidel); one LDS tile per workgroup.
#include "mg_kern.h"

namespace mg {
namespace {

// ---------------------------------------------------------------------------
// 2D smoothing sweep (one LDS tile per workgroup, no marching)
// ---------------------------------------------------------------------------

template <typename ST, int SM, bool VAR, int BY, int FL>
__global__ __launch_bounds__(NT) void k_smooth2d(const GridDesc* __restrict__ descs, int sel) {
    using T = arith_t<ST>;  // arithmetic type; ST is the storage type of u, f and the coarse correction
    static_assert(!VAR || sizeof(ST) == sizeof(T), "coefficient fields are stored in the arithmetic type");
    constexpr int flags = FL;
    // SWEEP_NORM: also sum r^2 of the incoming iterate over the tile's output nodes
    constexpr bool NRM = (FL & SWEEP_NORM) != 0;
    static_assert(!NRM || sizeof(T) == 8, "the sweep's norm sums FP64 residuals");
    const GridDesc d = descs[blockIdx.y];
    if (d.done && *gp(d.done)) return;
    constexpr int H = SM == SM_RBGS ? 2 : 1;
    constexpr int TX = BX - 2 * H, TY = BY - 2 * H, RPT = BY / 4;
    const int n = d.n;
    const int ntx = (n - 2 + TX - 1) / TX;
    const int tile = sweep_tile(sel, blockIdx.x, gridDim.x);
    const int x0 = 1 + (tile % ntx) * TX, y0 = 1 + (tile / ntx) * TY;
    const MG_GLOBAL ST* __restrict__ uin = gp((const ST*)((sel & 1) ? d.t : d.u));
    MG_GLOBAL ST* __restrict__ uout = gp((ST*)((sel & 1) ? d.u : d.t));
    const MG_GLOBAL ST* __restrict__ f = gp((const ST*)d.f);
    const MG_GLOBAL T* __restrict__ kf = gp((const T*)d.k);
    const MG_GLOBAL ST* __restrict__ ec = gp((const ST*)d.uc);
    const int nc = (n - 1) / 2 + 1;
    const T c = (T)d.c, wd = (T)d.wd, om = (T)d.omega;

    __shared__ T U[BY][BX];
    __shared__ T R[SM == SM_RBGS ? BY : 1][BX];
    __shared__ T K[VAR ? BY : 1][BX];

    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int gx = x0 - H + lane;
    const int cfirst = (sel & SEL_BLACK_FIRST) ? 1 : 0;  // colour of the first half-sweep
    const bool colg = gx >= 0 && gx < n, coli = gx >= 1 && gx <= n - 2;
    const bool lane1 = lane >= 1 && lane <= BX - 2;  // tile + 1 ring (RBGS) / tile (Jacobi)
    // Coarse-grid correction (bilinear, as interp2): each lane loads its
    // coarse column in the coarse rows y/2 and y/2 + (y odd) from clamped
    // addresses; an odd-x node takes the other coarse column from the
    // neighbouring lane.  x0 is odd, so with the two-node halo (RBGS) even
    // lanes hold odd x and their partner is the next lane (loaded at x/2), and
    // with the one-node halo (Jacobi) odd lanes hold odd x and their partner
    // is the previous lane (loaded at (x+1)/2): no lane needs one outside the
    // wavefront.
    const int xcl = min(max(gx, 0), n - 1);
    const int cx = H == 2 ? xcl >> 1 : (xcl + 1) >> 1;
    const bool xo = (gx & 1) != 0;
    T fr[RPT];
#pragma unroll
    for (int m = 0; m < RPT; ++m) {
        const int ly = w + 4 * m, gy = y0 - H + ly;
        const bool ing = colg && gy >= 0 && gy < n;
        const bool inn = coli && gy >= 1 && gy <= n - 2;
        const size_t p = (size_t)gy * n + gx;
        T v = T(0);
        if (ing && !(flags & SWEEP_ZERO_GUESS)) v = uin[p];
        if constexpr ((flags & SWEEP_PROLONG) != 0) {
            const int ycl = min(max(gy, 0), n - 1);
            const MG_GLOBAL ST* __restrict__ r0 = ec + (size_t)(ycl >> 1) * nc;
            const T a = r0[cx], b = r0[(ycl & 1) ? nc + cx : cx];
            T sa, sb;
            if constexpr (H == 2) {
                const T an = lane_next(a), bn = lane_next(b);  // every lane active
                sa = xo ? a + an : a;
                sb = xo ? b + bn : b;
            } else {
                const T ap = lane_prev(a), bp = lane_prev(b);
                sa = xo ? ap + a : a;
                sb = xo ? bp + b : b;
            }
            const T corr = (ycl & 1) ? (xo ? T(0.25) * (sa + sb) : T(0.5) * (sa + sb)) : (xo ? T(0.5) * sa : sa);
            if (inn) v = stored<ST>(v + corr);
        }
        U[ly][lane] = v;
        if constexpr (VAR) K[ly][lane] = ing ? kf[p] : T(1);
        fr[m] = (inn && lane1 && ly >= 1 && ly <= BY - 2) ? f[p] : T(0);
    }
    __syncthreads();
    [[maybe_unused]] double nacc = 0.0;
    if constexpr (SM == SM_RBGS) {
        // first colour (red unless black first) on the tile plus a one-node ring
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            const int ly = w + 4 * m, gy = y0 - H + ly;
            if (lane1 && ly >= 1 && ly <= BY - 2) {
                const bool inn = coli && gy >= 1 && gy <= n - 2;
                T v = U[ly][lane];
                if constexpr (NRM) {
                    // residual of both colours on the incoming values; summed over the output nodes
                    if (inn) {
                        T ds;
                        const T r = lds_res2<T, VAR>(U, K, ly, lane, fr[m], c, ds);
                        if (((gx + gy) & 1) == cfirst) v = stored<ST>(relax<T, VAR>(v, r, ds, c, wd, om));
                        if (lane >= 2 && lane <= BX - 3 && ly >= 2 && ly <= BY - 3 && gx <= n - 2 && gy <= n - 2)
                            nacc += r * r;
                    }
                } else {
                    if (inn && ((gx + gy) & 1) == cfirst) {
                        T ds;
                        const T r = lds_res2<T, VAR>(U, K, ly, lane, fr[m], c, ds);
                        v = stored<ST>(relax<T, VAR>(v, r, ds, c, wd, om));
                    }
                }
                R[ly][lane] = v;
            }
        }
        __syncthreads();
        // second colour on the tile, written out of place
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            const int ly = w + 4 * m, gy = y0 - H + ly;
            if (lane >= 2 && lane <= BX - 3 && ly >= 2 && ly <= BY - 3 && gx <= n - 2 && gy <= n - 2) {
                T v = R[ly][lane];
                if (((gx + gy) & 1) != cfirst) {
                    T ds;
                    const T r = lds_res2<T, VAR>(R, K, ly, lane, fr[m], c, ds);
                    v = relax<T, VAR>(v, r, ds, c, wd, om);
                }
                uout[(size_t)gy * n + gx] = (ST)v;
            }
        }
    } else {
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            const int ly = w + 4 * m, gy = y0 - H + ly;
            if (lane1 && ly >= 1 && ly <= BY - 2 && gx <= n - 2 && gy <= n - 2) {
                T ds;
                const T r = lds_res2<T, VAR>(U, K, ly, lane, fr[m], c, ds);
                if constexpr (NRM) nacc += r * r;
                uout[(size_t)gy * n + gx] = (ST)relax<T, VAR>(U[ly][lane], r, ds, c, wd, om);
            }
        }
    }
    if constexpr (NRM) {
        __shared__ double red4[4];
        const double tot = block_sum(nacc, red4);
        if (threadIdx.x == 0) gp(d.npart)[blockIdx.x] = tot;
    }
}

}  // namespace

template <typename T, int SMV, bool VARV, int FL>
hipError_t launch_smooth2d_fl(const GridDesc* d, int sel, TileCfg cfg, dim3 grid, hipStream_t s) {
    MG_BY_SWITCH(cfg.by, (k_smooth2d<T, SMV, VARV, BY, FL><<<grid, NT, 0, s>>>(d, sweep_arg(sel, cfg))))
    return hipSuccess;
}

template <typename T>
hipError_t launch_smooth2d(int sm, bool var, const GridDesc* d, int sel, int flags, TileCfg cfg, dim3 grid,
                           hipStream_t s) {
#define MG_FL(SMV, VARV)                                                                                   \
    switch (flags) {                                                                                       \
        case 0: return launch_smooth2d_fl<T, SMV, VARV, 0>(d, sel, cfg, grid, s);                           \
        case SWEEP_ZERO_GUESS: return launch_smooth2d_fl<T, SMV, VARV, SWEEP_ZERO_GUESS>(d, sel, cfg, grid, s); \
        case SWEEP_PROLONG: return launch_smooth2d_fl<T, SMV, VARV, SWEEP_PROLONG>(d, sel, cfg, grid, s);   \
        case SWEEP_NORM:                                                                                   \
            if constexpr (sizeof(T) == 8) return launch_smooth2d_fl<T, SMV, VARV, SWEEP_NORM>(d, sel, cfg, grid, s); \
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

template hipError_t launch_smooth2d<double>(int, bool, const GridDesc*, int, int, TileCfg, dim3, hipStream_t);
template hipError_t launch_smooth2d<float>(int, bool, const GridDesc*, int, int, TileCfg, dim3, hipStream_t);
template hipError_t launch_smooth2d<half_t>(int, bool, const GridDesc*, int, int, TileCfg, dim3, hipStream_t);

}  // namespace mg
