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

// ---------------------------------------------------------------------------
// 2D Laplacian: the first two red-black pre-smoothing sweeps of a level whose
// iterate starts at zero, in one launch.  A wavefront marches a strip of 128
// nodes (two per lane) along y through a chunk of rows; the four
// half-sweeps trail each other by one row (step kk: red of row kk from f,
// black of kk-1, red of kk-2, black of kk-3, which is written), each valid
// on the strip minus one more node per side, so a strip writes 122 nodes per
// row; y-neighbours come from five-row rings in registers, x-neighbours from
// the lane's other node and the adjacent lanes: no LDS, no barrier.  The four
// wavefronts of a workgroup take four consecutive chunks of one strip.  The
// expressions are those of the two separate sweeps (the first with every old
// value zero), stored values rounded to the storage type in between.
// ---------------------------------------------------------------------------
// Two adjacent nodes per lane (xa = xs + 2 lane, xb = xa + 1): the colour of
// the a-node of a row is the same on every lane, so each half-sweep updates
// exactly one node of every lane (a uniform choice); x-neighbours are the
// lane's other node and the adjacent lane's.
template <typename ST, int H>
struct PairRow {
    using T = arith_t<ST>;
    static constexpr int TX = 2 * BX - 2 * H;
    int n, xs, lane;
    unsigned ba, bb;   // byte offsets of the two nodes (clamped)
    bool ia, ib;       // the node is an inner node in x
    __device__ __forceinline__ void init() {
        const int xa = xs + 2 * lane;
        ba = (unsigned)min(max(xa, 0), n - 1) * (unsigned)sizeof(ST);
        bb = (unsigned)min(max(xa + 1, 0), n - 1) * (unsigned)sizeof(ST);
        ia = xa >= 1 && xa <= n - 2;
        ib = xa + 1 >= 1 && xa + 1 <= n - 2;
    }
    __device__ __forceinline__ const MG_GLOBAL ST* row(const MG_GLOBAL ST* p, int y) const {
        return p + (size_t)min(max(y, 0), n - 1) * n;
    }
    // node offsets 2 lane (a) and 2 lane + 1 (b) inside [q, 2 BX - 1 - q]
    template <int q>
    __device__ __forceinline__ bool va_ok() const { return 2 * lane >= q && 2 * lane <= 2 * BX - 1 - q; }
    template <int q>
    __device__ __forceinline__ bool vb_ok() const { return 2 * lane + 1 >= q && 2 * lane + 1 <= 2 * BX - 1 - q; }
    // half-sweep q of colour col on row y: (a, b) the row, (sa, sb) / (na, nb) the rows below / above
    template <int q>
    __device__ __forceinline__ void half(T& a, T& b, T sa, T sb, T na, T nb, T fa, T fb, int y, int col, T c, T wd,
                                         T om) const {
        const bool yin = y >= 1 && y <= n - 2;
        const T bw = lane_prev(b), an = lane_next(a);  // every lane active
        if (((xs + y) & 1) == col) {
            const T r = res_lap2(a, bw, b, sa, na, fa, c);
            const T nv = stored<ST>(relax<T, false>(a, r, T(0), c, wd, om));
            if (yin && ia && va_ok<q>()) a = nv;
        } else {
            const T r = res_lap2(b, a, an, sb, nb, fb, c);
            const T nv = stored<ST>(relax<T, false>(b, r, T(0), c, wd, om));
            if (yin && ib && vb_ok<q>()) b = nv;
        }
    }
};

template <typename ST>
struct Sweep2Row {
    using T = arith_t<ST>;
    static constexpr int H = 3, R = 5;
    using PR = PairRow<ST, H>;
    static constexpr int TX = PR::TX;
    PR pr;
    const MG_GLOBAL ST* __restrict__ f;
    MG_GLOBAL ST* __restrict__ uout;
    int n, y0, y1;
    T c, wd, om;
    T va[R], vb[R];   // latest values of rows kk-4 .. kk
    T fa[R], fb[R];   // f of rows kk-3 .. kk+1 (kk+1 in flight)

    template <int P>
    __device__ __forceinline__ void step(int kk) {
        constexpr int S0 = P, S1 = (P + 4) % R, S2 = (P + 3) % R, S3 = (P + 2) % R, S4 = (P + 1) % R;
        {
            const MG_GLOBAL ST* fr = pr.row(f, kk + 1);
            fa[S4] = ld_off(fr, pr.ba);
            fb[S4] = ld_off(fr, pr.bb);
        }
        {
            const T zero = T(0);
            const bool zin = kk >= 1 && kk <= n - 2;
            const T ra = res_lap2(zero, zero, zero, zero, zero, fa[S0], c);
            const T rb = res_lap2(zero, zero, zero, zero, zero, fb[S0], c);
            const T na = stored<ST>(relax<T, false>(zero, ra, zero, c, wd, om));
            const T nb = stored<ST>(relax<T, false>(zero, rb, zero, c, wd, om));
            const bool a_red = ((pr.xs + kk) & 1) == 0;
            va[S0] = (zin && pr.ia && a_red) ? na : zero;
            vb[S0] = (zin && pr.ib && !a_red) ? nb : zero;
        }
        if (kk - 1 >= y0 - 2)
            pr.template half<1>(va[S1], vb[S1], va[S2], vb[S2], va[S0], vb[S0], fa[S1], fb[S1], kk - 1, 1, c, wd, om);
        if (kk - 2 >= y0 - 1)
            pr.template half<2>(va[S2], vb[S2], va[S3], vb[S3], va[S1], vb[S1], fa[S2], fb[S2], kk - 2, 0, c, wd, om);
        const int y3 = kk - 3;
        if (y3 >= y0 && y3 < y1) {
            pr.template half<3>(va[S3], vb[S3], va[S4], vb[S4], va[S2], vb[S2], fa[S3], fb[S3], y3, 1, c, wd, om);
            if (y3 >= 1 && y3 <= n - 2) {
                MG_GLOBAL ST* o = uout + (size_t)y3 * n;
                if (pr.ia && pr.template va_ok<H>()) st_off(o, pr.ba, (ST)va[S3]);
                if (pr.ib && pr.template vb_ok<H>()) st_off(o, pr.bb, (ST)vb[S3]);
            }
        }
    }
    __device__ __forceinline__ void run() {
        pr.init();
#pragma unroll
        for (int q = 0; q < R; ++q) va[q] = vb[q] = fa[q] = fb[q] = T(0);
        int kk = y0 - H;
        const int kend = y1 - 1 + H;
        {
            const MG_GLOBAL ST* fr = pr.row(f, kk);
            fa[0] = ld_off(fr, pr.ba);
            fb[0] = ld_off(fr, pr.bb);
        }
        for (; kk + 4 <= kend; kk += R) {
            step<0>(kk);
            step<1>(kk + 1);
            step<2>(kk + 2);
            step<3>(kk + 3);
            step<4>(kk + 4);
        }
        if (kk <= kend) step<0>(kk);
        if (kk + 1 <= kend) step<1>(kk + 1);
        if (kk + 2 <= kend) step<2>(kk + 2);
        if (kk + 3 <= kend) step<3>(kk + 3);
    }
};

template <typename ST>
__global__ __launch_bounds__(NT) void k_smooth2d_zg2(const GridDesc* __restrict__ descs, int sel, int ychunk) {
    const GridDesc d = descs[blockIdx.y];
    if (d.done && *gp(d.done)) return;
    using S = Sweep2Row<ST>;
    using T = arith_t<ST>;
    S s;
    const int n = d.n;
    const int ntx = (n - 2 + S::TX - 1) / S::TX;
    const int tile = sweep_tile(sel, blockIdx.x, gridDim.x);
    const int tx = tile % ntx, tb = tile / ntx;
    const int w = threadIdx.x >> 6;
    s.n = n;
    s.pr.n = n;
    s.pr.lane = threadIdx.x & 63;
    s.pr.xs = 1 + tx * S::TX - S::H;
    s.y0 = min(1 + (tb * 4 + w) * ychunk, n - 1);
    s.y1 = min(s.y0 + ychunk, n - 1);
    if (s.y0 >= s.y1) return;  // a wavefront past the last chunk (no barrier follows)
    s.uout = gp((ST*)((sel & 1) ? d.u : d.t));
    s.f = gp((const ST*)d.f);
    s.c = (T)d.c;
    s.wd = (T)d.wd;
    s.om = (T)d.omega;
    s.run();
}

// ---------------------------------------------------------------------------
// 2D Laplacian: the first two red-black post-smoothing sweeps in one launch,
// the first with the coarse-grid correction (Algorithm 1: interpolation and
// correction, postsmoothing) added as each row enters.  A wavefront marches
// a strip of 128 nodes (two per lane) along y through a chunk of rows: step
// kk corrects row kk (u + P uc at inner nodes, the bilinear weights of the
// separate sweep), the first colour of row kk-1, the second of kk-2, the
// first of kk-3 and the second of kk-4, which it writes to the ping-pong
// partner of its input.  The half-sweeps are valid one node narrower per
// side each, so a strip writes 120 nodes per row; six-row register rings
// hold every node's latest value and f.  Colours follow the select's
// black-first bit (the symmetric smoother relaxes black first after the
// correction).
// ---------------------------------------------------------------------------
template <typename ST>
struct Sweep2Pro {
    using T = arith_t<ST>;
    static constexpr int H = 4, R = 6;
    using PR = PairRow<ST, H>;
    static constexpr int TX = PR::TX;
    PR pr;
    const MG_GLOBAL ST* __restrict__ uin;
    MG_GLOBAL ST* __restrict__ uout;
    const MG_GLOBAL ST* __restrict__ f;
    const MG_GLOBAL ST* __restrict__ ec;
    int n, nc, y0, y1, cfirst;
    unsigned cbb;  // byte offset of the coarse column of the b-node (xs odd: b is even, a = b - 1 is odd)
    unsigned cab;  // byte offset of the coarse column left of the a-node
    T c, wd, om;
    T va[R], vb[R];   // latest values of rows kk-5 .. kk
    T fa[R], fb[R];   // f of rows kk-4 .. kk+1 (kk+1 in flight)
    T ua, ub;         // u of row kk+1 (in flight)

    // (a, b) += P uc at row y (bilinear, as the separate sweep; inner nodes only)
    __device__ __forceinline__ void correct(T& a, T& b, int y) const {
        const int ycl = min(max(y, 0), n - 1);
        const MG_GLOBAL ST* __restrict__ r0 = ec + (size_t)(ycl >> 1) * nc;
        const MG_GLOBAL ST* __restrict__ r1 = r0 + ((ycl & 1) ? nc : 0);
        const T c0 = ld_off(r0, cbb), c1 = ld_off(r1, cbb);  // column of b (and right of a)
        const T p0 = ld_off(r0, cab), p1 = ld_off(r1, cab);  // column left of a
        // a (odd x): the coarse columns left and right; b (even x): its own column
        const T sa0 = p0 + c0, sa1 = p1 + c1;
        const T ca = (ycl & 1) ? T(0.25) * (sa0 + sa1) : T(0.5) * sa0;
        const T cb = (ycl & 1) ? T(0.5) * (c0 + c1) : c0;
        const bool yin = y >= 1 && y <= n - 2;
        if (yin && pr.ia) a = stored<ST>(a + ca);
        if (yin && pr.ib) b = stored<ST>(b + cb);
    }
    template <int P>
    __device__ __forceinline__ void step(int kk) {
        constexpr int S0 = P, S1 = (P + 5) % R, S2 = (P + 4) % R, S3 = (P + 3) % R, S4 = (P + 2) % R,
                      S5 = (P + 1) % R;
        const int c1 = cfirst, c2 = cfirst ^ 1;
        va[S0] = ua;
        vb[S0] = ub;
        correct(va[S0], vb[S0], kk);
        {
            const MG_GLOBAL ST* ur = pr.row(uin, kk + 1);
            ua = ld_off(ur, pr.ba);
            ub = ld_off(ur, pr.bb);
            const MG_GLOBAL ST* fr = pr.row(f, kk + 1);
            fa[S5] = ld_off(fr, pr.ba);  // slot of row kk-5, whose f is no longer read
            fb[S5] = ld_off(fr, pr.bb);
        }
        if (kk - 1 >= y0 - 3)
            pr.template half<1>(va[S1], vb[S1], va[S2], vb[S2], va[S0], vb[S0], fa[S1], fb[S1], kk - 1, c1, c, wd, om);
        if (kk - 2 >= y0 - 2)
            pr.template half<2>(va[S2], vb[S2], va[S3], vb[S3], va[S1], vb[S1], fa[S2], fb[S2], kk - 2, c2, c, wd, om);
        if (kk - 3 >= y0 - 1)
            pr.template half<3>(va[S3], vb[S3], va[S4], vb[S4], va[S2], vb[S2], fa[S3], fb[S3], kk - 3, c1, c, wd, om);
        const int y4 = kk - 4;
        if (y4 >= y0 && y4 < y1) {
            pr.template half<4>(va[S4], vb[S4], va[S5], vb[S5], va[S3], vb[S3], fa[S4], fb[S4], y4, c2, c, wd, om);
            if (y4 >= 1 && y4 <= n - 2) {
                MG_GLOBAL ST* o = uout + (size_t)y4 * n;
                if (pr.ia && pr.template va_ok<H>()) st_off(o, pr.ba, (ST)va[S4]);
                if (pr.ib && pr.template vb_ok<H>()) st_off(o, pr.bb, (ST)vb[S4]);
            }
        }
    }
    __device__ __forceinline__ void run() {
        pr.init();
        const int xb = pr.xs + 2 * pr.lane + 1;
        cbb = (unsigned)(min(max(xb, 0), n - 1) >> 1) * (unsigned)sizeof(ST);
        cab = (unsigned)(min(max(xb - 2, 0), n - 1) >> 1) * (unsigned)sizeof(ST);
#pragma unroll
        for (int q = 0; q < R; ++q) va[q] = vb[q] = fa[q] = fb[q] = T(0);
        int kk = y0 - H;
        const int kend = y1 - 1 + H;
        {
            const MG_GLOBAL ST* ur = pr.row(uin, kk);
            ua = ld_off(ur, pr.ba);
            ub = ld_off(ur, pr.bb);
            const MG_GLOBAL ST* fr = pr.row(f, kk);
            fa[0] = ld_off(fr, pr.ba);
            fb[0] = ld_off(fr, pr.bb);
        }
        for (; kk + 5 <= kend; kk += R) {
            step<0>(kk);
            step<1>(kk + 1);
            step<2>(kk + 2);
            step<3>(kk + 3);
            step<4>(kk + 4);
            step<5>(kk + 5);
        }
        if (kk <= kend) step<0>(kk);
        if (kk + 1 <= kend) step<1>(kk + 1);
        if (kk + 2 <= kend) step<2>(kk + 2);
        if (kk + 3 <= kend) step<3>(kk + 3);
        if (kk + 4 <= kend) step<4>(kk + 4);
    }
};

template <typename ST>
__global__ __launch_bounds__(NT) void k_smooth2d_pro2(const GridDesc* __restrict__ descs, int sel, int ychunk) {
    const GridDesc d = descs[blockIdx.y];
    if (d.done && *gp(d.done)) return;
    using S = Sweep2Pro<ST>;
    using T = arith_t<ST>;
    S s;
    const int n = d.n;
    const int ntx = (n - 2 + S::TX - 1) / S::TX;
    const int tile = sweep_tile(sel, blockIdx.x, gridDim.x);
    const int tx = tile % ntx, tb = tile / ntx;
    const int w = threadIdx.x >> 6;
    s.n = n;
    s.nc = (n - 1) / 2 + 1;
    s.pr.n = n;
    s.pr.lane = threadIdx.x & 63;
    s.pr.xs = 1 + tx * S::TX - S::H;  // odd
    s.y0 = min(1 + (tb * 4 + w) * ychunk, n - 1);
    s.y1 = min(s.y0 + ychunk, n - 1);
    if (s.y0 >= s.y1) return;  // a wavefront past the last chunk (no barrier follows)
    s.cfirst = (sel & SEL_BLACK_FIRST) ? 1 : 0;
    s.uin = gp((const ST*)((sel & 1) ? d.t : d.u));
    s.uout = gp((ST*)((sel & 1) ? d.u : d.t));
    s.f = gp((const ST*)d.f);
    s.ec = gp((const ST*)d.uc);
    s.c = (T)d.c;
    s.wd = (T)d.wd;
    s.om = (T)d.omega;
    s.run();
}

}  // namespace

int smooth2d_pro2_tiles(int n, int ychunk) {
    const int m = n - 2;
    return cdiv(m, 2 * BX - 8) * cdiv(cdiv(m, ychunk), 4);
}

template <typename T>
hipError_t launch_smooth2d_pro2(const GridDesc* d, int ninst, int n, int sel, TileCfg cfg, hipStream_t s) {
    if constexpr (sizeof(T) == 8) {
        return hipErrorInvalidValue;  // built for FP32 and binary16 storage
    } else {
        if (n < 5 || ninst <= 0 || cfg.zchunk < 1) return hipErrorInvalidValue;
        const dim3 grid(smooth2d_pro2_tiles(n, cfg.zchunk), ninst);
        k_smooth2d_pro2<T><<<grid, NT, 0, s>>>(d, sweep_arg(sel, cfg), cfg.zchunk);
        return hipGetLastError();
    }
}
template hipError_t launch_smooth2d_pro2<double>(const GridDesc*, int, int, int, TileCfg, hipStream_t);
template hipError_t launch_smooth2d_pro2<float>(const GridDesc*, int, int, int, TileCfg, hipStream_t);
template hipError_t launch_smooth2d_pro2<half_t>(const GridDesc*, int, int, int, TileCfg, hipStream_t);

int smooth2d_zg2_tiles(int n, int ychunk) {
    const int m = n - 2;
    return cdiv(m, 2 * BX - 6) * cdiv(cdiv(m, ychunk), 4);
}

template <typename T>
hipError_t launch_smooth2d_zg2(const GridDesc* d, int ninst, int n, int sel, TileCfg cfg, hipStream_t s) {
    if constexpr (sizeof(T) == 8) {
        return hipErrorInvalidValue;  // built for FP32 and binary16 storage
    } else {
        if (n < 5 || ninst <= 0 || cfg.zchunk < 1) return hipErrorInvalidValue;
        const dim3 grid(smooth2d_zg2_tiles(n, cfg.zchunk), ninst);
        k_smooth2d_zg2<T><<<grid, NT, 0, s>>>(d, sweep_arg(sel, cfg), cfg.zchunk);
        return hipGetLastError();
    }
}
template hipError_t launch_smooth2d_zg2<double>(const GridDesc*, int, int, int, TileCfg, hipStream_t);
template hipError_t launch_smooth2d_zg2<float>(const GridDesc*, int, int, int, TileCfg, hipStream_t);
template hipError_t launch_smooth2d_zg2<half_t>(const GridDesc*, int, int, int, TileCfg, hipStream_t);

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
