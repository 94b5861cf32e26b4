// FP64 residual norms, the FP64 refinement pass, device-side solve control and setup kernels.
#include "mg_kern.h"

namespace mg {
namespace {

// ---------------------------------------------------------------------------
// FP64 residual norm partials (solve loop of the Layer-4 Application function)
// ---------------------------------------------------------------------------

template <bool VAR, int BY>
__global__ __launch_bounds__(NT) void k_norm2d(const GridDesc* __restrict__ descs, int sel, double* __restrict__ part,
                                               int pstride) {
    const GridDesc d = descs[blockIdx.y];
    __shared__ double red4[4];
    if (d.done && *gp(d.done)) return;
    constexpr int TX = BX - 2, TY = BY - 2, RPT = BY / 4;
    const int n = d.n;
    const int ntx = (n - 2 + TX - 1) / TX;
    const int tile = blockIdx.x;
    const int x0 = 1 + (tile % ntx) * TX, y0 = 1 + (tile / ntx) * TY;
    const MG_GLOBAL double* __restrict__ u = gp((const double*)(sel ? d.t : d.u));
    const MG_GLOBAL double* __restrict__ f = gp((const double*)d.f);
    const MG_GLOBAL double* __restrict__ kf = gp((const double*)d.k);
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

// 3D residual of the FP64 finest level, marching along z.  IR selects the
// refinement variant: the plane entering the ring is u_in + e (inner nodes),
// its owned part is written to u_out, and r is stored in FP32.  WV wavefronts
// per workgroup; a thread holds rows w, w + WV, ... of the tile.
template <bool VAR, int BY, int PD, bool IR, int WV>
struct Resid3D {
    static constexpr int TX = BX - 2, TY = BY - 2, RPT = BY / WV;
    static_assert(RPT >= 1 && RPT * WV == BY, "tile rows must be a multiple of the wavefronts");
    double (*U)[BY][BX];
    double (*K)[BY][BX];
    const MG_GLOBAL double* __restrict__ uin;
    MG_GLOBAL double* __restrict__ uout;
    const MG_GLOBAL float* __restrict__ e;
    const MG_GLOBAL double* __restrict__ f;
    const MG_GLOBAL double* __restrict__ kf;
    MG_GLOBAL float* __restrict__ r32;
    int n, x0, y0, z0, z1, kstart, kend, flags;
    double c;
    int lane, w, gx;
    bool coli, lane1;
    double un[3][RPT], kn[3][RPT], fr[3][RPT];
    double uo[3][RPT], ko[3][RPT];  // plane values (u + e) and k at own positions, planes kk, kk-1, kk-2
    float en[3][RPT];
    double acc = 0.0;

    __device__ __forceinline__ int gy(int m) const { return y0 - 1 + w + WV * m; }

    // Rows are wave-uniform (the wave index is read into a scalar register):
    // each row of a plane has a scalar base address and the per-lane part is
    // the byte offset of the lane's clamped x position (xb for 8-byte words,
    // xb4 for the FP32 correction and residual).
    unsigned xb, xb4;
    unsigned minner, mring;
    size_t pl;

    __device__ __forceinline__ int rowoff(int m) const { return min(max(gy(m), 0), n - 1) * n; }

    __device__ __forceinline__ void init_rows() {
        pl = (size_t)n * n;
        const int xc = min(max(gx, 0), n - 1);
        xb = (unsigned)xc * 8u;
        xb4 = (unsigned)xc * 4u;
        minner = mring = 0;
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            const int y = gy(m), ly = w + WV * m;
            if (coli && y >= 1 && y <= n - 2) minner |= 1u << m;
            if (lane1 && ly >= 1 && ly <= BY - 2) mring |= 1u << m;
        }
    }

    // Unconditional loads from clamped (always in-bounds) addresses, kept as
    // loaded: a value at a position outside the grid or off the inner nodes is
    // never used, since every residual and update is taken at an inner node,
    // whose neighbours all lie in the grid.  No select on the loaded value, so
    // no branch around the loads and no wait for them before they are used.
    __device__ __forceinline__ void issue(int z, double (&du)[RPT], float (&de)[RPT], double (&dk)[RPT]) {
        const size_t zoff = (size_t)min(max(z, 0), n - 1) * pl;
        const MG_GLOBAL double* __restrict__ up = uin + zoff;
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            du[m] = ld_off(up + rowoff(m), xb);
            if constexpr (IR) {
                if (!(flags & IR_NO_UPDATE)) de[m] = ld_off(e + zoff + rowoff(m), xb4);
                else de[m] = 0.0f;
            }
            if constexpr (VAR) dk[m] = ld_off(kf + zoff + rowoff(m), xb);
        }
    }
    // f is read on the tile rows only (the halo rows have no residual).
    __device__ __forceinline__ void issue_f(int z, double (&dst)[RPT]) {
        const MG_GLOBAL double* __restrict__ fp = f + (size_t)min(max(z, 0), n - 1) * pl;
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            const int ly = w + WV * m;  // wave-uniform
            if (ly >= 1 && ly <= BY - 2) dst[m] = ld_off(fp + rowoff(m), xb);
        }
    }

    template <int P>
    __device__ __forceinline__ void step(int kk) {
        constexpr int S0 = P, S1 = (P + 2) % 3, S2 = (P + 1) % 3, SN = (P + PD) % 3;
        const bool zin = kk >= 1 && kk <= n - 2;
        const bool own = kk >= z0 && kk < z1;
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            const int ly = w + WV * m, y = gy(m);
            double v = un[S0][m];
            if constexpr (IR) {
                const bool inn = zin && coli && y >= 1 && y <= n - 2;
                if (inn && !(flags & IR_NO_UPDATE)) {
                    v = v + (double)en[S0][m];
                    if (own && ((mring >> m) & 1u)) st_off(uout + (size_t)kk * pl + rowoff(m), xb, v);
                }
            }
            uo[S0][m] = v;
            U[S0][ly][lane] = v;
            if constexpr (VAR) {
                ko[S0][m] = kn[S0][m];
                K[S0][ly][lane] = kn[S0][m];
            }
        }
        // f of the plane PD - 1 ahead: with PD = 2 into the slot of plane
        // kk-2, whose f had its last use in the previous step
        if constexpr (PD == 2) issue_f(kk + 1, fr[S2]);
        else issue_f(kk, fr[S0]);
        issue(kk + PD, un[SN], en[SN], kn[SN]);
        __syncthreads();
        // residual of plane kk-1: z-neighbours from registers, x from the
        // adjacent lanes, y from LDS (slot S1 is rewritten two steps later,
        // after the next barrier)
        const int zz = kk - 1;
        if (zz >= z0) {
#pragma unroll
            for (int m = 0; m < RPT; ++m) {
                const int ly = w + WV * m;
                const double uc = uo[S1][m];
                const double uw = lane_prev(uc), ue = lane_next(uc);
                double kc = 1.0, kw = 1.0, ke = 1.0, kb = 1.0, ka = 1.0, kS = 1.0, kN = 1.0;
                if constexpr (VAR) {
                    kc = ko[S1][m];
                    kw = lane_prev(kc);
                    ke = lane_next(kc);
                    kb = ko[S2][m];
                    ka = ko[S0][m];
                }
                if ((mring >> m) & (minner >> m) & 1u) {
                    if constexpr (VAR) {
                        kS = K[S1][ly - 1][lane];
                        kN = K[S1][ly + 1][lane];
                    }
                    double ds;
                    const double r = res3<double, VAR>(uc, uw, ue, U[S1][ly - 1][lane], U[S1][ly + 1][lane],
                                                       uo[S2][m], uo[S0][m], kc, kw, ke, kS, kN, kb, ka, fr[S1][m],
                                                       c, ds);
                    if constexpr (IR) st_off(r32 + (size_t)zz * pl + rowoff(m), xb4, (float)r);
                    acc += r * r;
                }
            }
        }
    }

    __device__ __forceinline__ void run() {
        init_rows();
        int kk = kstart;
#pragma unroll
        for (int m = 0; m < RPT; ++m) fr[0][m] = fr[1][m] = fr[2][m] = 0.0;  // halo rows: f is not read
        issue(kk, un[0], en[0], kn[0]);
        if constexpr (PD == 2) {
            issue(kk + 1, un[1], en[1], kn[1]);
            issue_f(kk, fr[0]);
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

template <bool VAR, int BY, int PD, bool IR, int WV>
__device__ __forceinline__ void resid3d_body(const GridDesc* gd, const IRDesc* ird, int sel, int flags,
                                             double* __restrict__ part, int pstride, int zchunk) {
    using S = Resid3D<VAR, BY, PD, IR, WV>;
    __shared__ double red[WV];
    __shared__ double U[3][BY][BX];
    __shared__ double K[VAR ? 3 : 1][BY][BX];
    S s;
    int n, inst;
    if constexpr (IR) {
        const IRDesc d = *ird;
        if (d.par) sel = *gp(d.par);
        n = d.n;
        inst = d.inst;
        s.uin = gp((const double*)(sel ? d.u[1] : d.u[0]));  // a select: indexing the copy would spill it
        s.uout = gp(sel ? d.u[0] : d.u[1]);
        s.e = gp((const float*)d.e);
        s.f = gp(d.f);
        s.kf = gp(d.k);
        s.r32 = gp((float*)d.r);
        s.c = d.c;
    } else {
        const GridDesc d = *gd;
        n = d.n;
        inst = d.inst;
        s.uin = gp((const double*)(sel ? d.t : d.u));
        s.uout = nullptr;
        s.e = nullptr;
        s.f = gp((const double*)d.f);
        s.kf = gp((const double*)d.k);
        s.r32 = nullptr;
        s.c = d.c;
    }
    s.U = U;
    s.K = K;
    const int ntx = (n - 2 + S::TX - 1) / S::TX, nty = (n - 2 + S::TY - 1) / S::TY;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int tx = tile % ntx, t2 = tile / ntx, ty = t2 % nty, tz = t2 / nty;
    s.n = n;
    s.x0 = 1 + tx * S::TX;
    s.y0 = 1 + ty * S::TY;
    s.z0 = 1 + tz * zchunk;
    s.z1 = min(s.z0 + zchunk, n - 1);
    s.kstart = s.z0 - 1;
    s.kend = s.z1;
    s.flags = flags;
    s.lane = threadIdx.x & 63;
    s.w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    s.gx = s.x0 - 1 + s.lane;
    s.coli = s.gx >= 1 && s.gx <= n - 2;
    s.lane1 = s.lane >= 1 && s.lane <= BX - 2;
    s.run();
    const double t = block_sum_w<WV>(s.acc, red);
    if (threadIdx.x == 0) part[(size_t)inst * pstride + blockIdx.x] = t;
}

// Paired variant of the 3D pass (Laplacian): a lane owns two adjacent nodes
// of a box row, a at odd x and b = a + 1, so a wavefront computes 128 nodes of
// a row and every load and store of a pair moves 16 bytes (FP64) or 8 bytes
// (FP32).  The inner nodes 1 .. n-2 of a row (n-2 = 2^L - 1) split into whole
// 128-node tiles; pairs (x, x+1) with odd x never cross the row's end (the
// last is (n-2, n-1)), and pairs of lanes past the grid are clamped onto it.
// The two x-neighbours outside the box (x0-1 for lane 0, x0+128 for lane 63)
// are loaded on their own, one word per row.  The update and residual take the
// same values and the same per-point expressions as the one-node-per-lane pass.
// Pairs are accessed field by field through pointers of the word's own
// alignment; the compiler merges them into one 16- or 8-byte access.
struct __attribute__((aligned(8))) Dbl2 {
    double a, b;
};
struct __attribute__((aligned(4))) Flt2 {
    float a, b;
};
struct __attribute__((aligned(2))) Hlf2 {
    half_t a, b;
};
// pair type of the correction / residual words
template <typename E>
struct PairOf {
    using type = Flt2;
};
template <>
struct PairOf<half_t> {
    using type = Hlf2;
};
__device__ __forceinline__ Dbl2 ld_d2(const MG_GLOBAL double* base, unsigned boff) {
    const MG_GLOBAL Dbl2* q = (const MG_GLOBAL Dbl2*)((const MG_GLOBAL char*)base + boff);
    Dbl2 v;
    v.a = q->a;
    v.b = q->b;
    return v;
}
template <typename E>
__device__ __forceinline__ typename PairOf<E>::type ld_f2(const MG_GLOBAL E* base, unsigned boff) {
    using P2 = typename PairOf<E>::type;
    const MG_GLOBAL P2* q = (const MG_GLOBAL P2*)((const MG_GLOBAL char*)base + boff);
    P2 v;
    v.a = q->a;
    v.b = q->b;
    return v;
}
__device__ __forceinline__ void st_d2(MG_GLOBAL double* base, unsigned boff, const Dbl2& v) {
    MG_GLOBAL Dbl2* q = (MG_GLOBAL Dbl2*)((MG_GLOBAL char*)base + boff);
    q->a = v.a;
    q->b = v.b;
}
template <typename E>
__device__ __forceinline__ void st_f2(MG_GLOBAL E* base, unsigned boff, const typename PairOf<E>::type& v) {
    using P2 = typename PairOf<E>::type;
    MG_GLOBAL P2* q = (MG_GLOBAL P2*)((MG_GLOBAL char*)base + boff);
    q->a = v.a;
    q->b = v.b;
}

// Half-precision form: the scale for a residual of largest magnitude mx, the
// power of two s with 8 <= s mx < 16, its exponent kept in [-126, 127] so that
// s is a normal float (1 for zero or non-finite mx).
__device__ __forceinline__ double fp16_scale(double mx) {
    if (!(mx > 0.0) || !(mx <= 1.7976931348623157e308)) return 1.0;
    int e;
    (void)frexp(mx, &e);  // mx = m 2^e, 1/2 <= m < 1
    return ldexp(1.0, min(127, max(-126, 4 - e)));
}

// Correction word -> FP64 increment, residual -> stored word: plain
// conversions for float words; binary16 words carry the power-of-two scale
// (the increment e / s_e, the stored residual half(float(s_r) * float(r))).
template <typename E>
struct IRWords {
    double inv = 1.0;  // 1 / scale of the correction read
    float sr = 1.0f;   // scale of the residual written
    __device__ __forceinline__ double incr(E x) const {
        if constexpr (sizeof(E) == 4) return (double)x;
        else return (double)(float)x * inv;
    }
    __device__ __forceinline__ E res(double r) const {
        if constexpr (sizeof(E) == 4) return (float)r;
        else return (E)(sr * (float)r);
    }
};

// Deterministic workgroup maximum (result valid in thread 0).
template <int WV>
__device__ __forceinline__ double block_max_w(double v, double* red) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    const int w = threadIdx.x >> 6;
    __syncthreads();  // red may still be read by the preceding block sum
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double m = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < WV; ++i) m = fmax(m, red[i]);
    return m;
}

template <int BY, int PD, bool IR, int WV, typename E = float>
struct Pair3D {
    static constexpr int TX = 2 * BX, TY = BY - 2, RPT = BY / WV;
    static_assert(RPT >= 1 && RPT * WV == BY, "tile rows must be a multiple of the wavefronts");
    using E2 = typename PairOf<E>::type;
    static constexpr bool H16 = sizeof(E) == 2;
    Dbl2 (*U)[BY][BX];
    const MG_GLOBAL double* __restrict__ uin;
    MG_GLOBAL double* __restrict__ uout;
    const MG_GLOBAL E* __restrict__ e;
    const MG_GLOBAL double* __restrict__ f;
    MG_GLOBAL E* __restrict__ r32;
    IRWords<E> wd;
    int n, x0, y0, z0, z1, kstart, kend, flags;
    double c;
    int lane, w;
    unsigned inx;     // bit 0: a inner in x, bit 1: b inner in x
    bool hin;         // the lane's outside neighbour (lane 0: x0-1, lane 63: x0+128) is an inner node
    unsigned xp8, xp4, xh8, xh4;  // byte offsets: the pair, the outside neighbour (8-byte / correction words)
    unsigned minner, mring;       // bit m: row m inner in y / in the tile rows 1 .. BY-2
    size_t pl;
    Dbl2 un[3][RPT], fr[3][RPT], uo[3][RPT];
    E2 en[3][RPT];
    double hn[3][RPT], ho[3][RPT];  // outside neighbour: as loaded / updated
    E he[3][RPT];
    double acc = 0.0;
    double mxr = 0.0;  // half-precision form: largest |r|

    __device__ __forceinline__ int gy(int m) const { return y0 - 1 + w + WV * m; }
    __device__ __forceinline__ int rowoff(int m) const { return min(max(gy(m), 0), n - 1) * n; }

    __device__ __forceinline__ void init_rows() {
        pl = (size_t)n * n;
        const int xa = x0 + 2 * lane;  // >= 1
        inx = (xa <= n - 2 ? 1u : 0u) | (xa + 1 <= n - 2 ? 2u : 0u);
        const unsigned xp = (unsigned)min(xa, n - 2);
        xp8 = xp * 8u;
        xp4 = xp * (unsigned)sizeof(E);
        // lanes 0 .. 31 read the left neighbour of the box, 32 .. 63 the right
        // one (clamped into the row); only lanes 0 and 63 use them
        const int xl = x0 - 1, xr = min(x0 + TX, n - 1);
        const unsigned xh = (unsigned)(lane < 32 ? xl : xr);
        xh8 = xh * 8u;
        xh4 = xh * (unsigned)sizeof(E);
        hin = lane == 0 ? xl >= 1 : (x0 + TX <= n - 2);
        minner = mring = 0;
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            const int y = gy(m), ly = w + WV * m;
            if (y >= 1 && y <= n - 2) minner |= 1u << m;
            if (ly >= 1 && ly <= BY - 2) mring |= 1u << m;
        }
    }

    __device__ __forceinline__ void issue(int z, Dbl2 (&du)[RPT], E2 (&de)[RPT], double (&dh)[RPT],
                                          E (&dhe)[RPT]) {
        const size_t zoff = (size_t)min(max(z, 0), n - 1) * pl;
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            const MG_GLOBAL double* row = uin + zoff + rowoff(m);
            du[m] = ld_d2(row, xp8);
            dh[m] = ld_off(row, xh8);
            if constexpr (IR) {
                if (!(flags & IR_NO_UPDATE)) {
                    const MG_GLOBAL E* erow = e + zoff + rowoff(m);
                    de[m] = ld_f2(erow, xp4);
                    dhe[m] = ld_off(erow, xh4);
                } else {
                    de[m] = E2{(E)0, (E)0};
                    dhe[m] = (E)0;
                }
            }
        }
    }
    // f on the tile rows only
    __device__ __forceinline__ void issue_f(int z, Dbl2 (&dst)[RPT]) {
        const MG_GLOBAL double* __restrict__ fp = f + (size_t)min(max(z, 0), n - 1) * pl;
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            const int ly = w + WV * m;  // wave-uniform
            if (ly >= 1 && ly <= BY - 2) dst[m] = ld_d2(fp + rowoff(m), xp8);
        }
    }

    template <int P>
    __device__ __forceinline__ void step(int kk) {
        constexpr int S0 = P, S1 = (P + 2) % 3, S2 = (P + 1) % 3, SN = (P + PD) % 3;
        const bool zin = kk >= 1 && kk <= n - 2;
        const bool own = kk >= z0 && kk < z1;
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            const int ly = w + WV * m;
            Dbl2 v = un[S0][m];
            double h = hn[S0][m];
            if constexpr (IR) {
                if (!(flags & IR_NO_UPDATE)) {
                    const bool iny = zin && ((minner >> m) & 1u);
                    if (iny && (inx & 1u)) v.a = v.a + wd.incr(en[S0][m].a);
                    if (iny && (inx & 2u)) v.b = v.b + wd.incr(en[S0][m].b);
                    if (iny && hin) h = h + wd.incr(he[S0][m]);
                    if (own && iny && ((mring >> m) & 1u)) {
                        MG_GLOBAL double* row = uout + (size_t)kk * pl + rowoff(m);
                        if (inx == 3u) st_d2(row, xp8, v);
                        else if (inx & 1u) st_off(row, xp8, v.a);
                    }
                }
            }
            uo[S0][m] = v;
            ho[S0][m] = h;
            U[S0][ly][lane] = v;
        }
        if constexpr (PD == 2) issue_f(kk + 1, fr[S2]);
        else issue_f(kk, fr[S0]);
        issue(kk + PD, un[SN], en[SN], hn[SN], he[SN]);
        __syncthreads();
        const int zz = kk - 1;
        if (zz >= z0) {
#pragma unroll
            for (int m = 0; m < RPT; ++m) {
                const int ly = w + WV * m;
                const Dbl2 uc = uo[S1][m];
                double wa = lane_prev(uc.b), eb = lane_next(uc.a);  // every lane active
                if (lane == 0) wa = ho[S1][m];
                if (lane == BX - 1) eb = ho[S1][m];
                if (((mring >> m) & (minner >> m) & 1u)) {
                    const Dbl2 dn = U[S1][ly - 1][lane], up = U[S1][ly + 1][lane];
                    const double ra = res_lap3<double>(uc.a, wa, uc.b, dn.a, up.a, uo[S2][m].a, uo[S0][m].a,
                                                       fr[S1][m].a, c);
                    const double rb = res_lap3<double>(uc.b, uc.a, eb, dn.b, up.b, uo[S2][m].b, uo[S0][m].b,
                                                       fr[S1][m].b, c);
                    if constexpr (IR) {
                        MG_GLOBAL E* row = r32 + (size_t)zz * pl + rowoff(m);
                        const E2 rv{wd.res(ra), wd.res(rb)};
                        if (inx == 3u) st_f2(row, xp4, rv);
                        else if (inx & 1u) st_off(row, xp4, rv.a);
                    }
                    if (inx & 1u) acc += ra * ra;
                    if (inx & 2u) acc += rb * rb;
                    if constexpr (H16) {
                        if (inx & 1u) mxr = fmax(mxr, fabs(ra));
                        if (inx & 2u) mxr = fmax(mxr, fabs(rb));
                    }
                }
            }
        }
    }

    __device__ __forceinline__ void run() {
        init_rows();
        int kk = kstart;
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
            fr[0][m] = fr[1][m] = fr[2][m] = Dbl2{0.0, 0.0};
            uo[1][m] = uo[2][m] = Dbl2{0.0, 0.0};
            ho[1][m] = ho[2][m] = 0.0;
        }
        issue(kk, un[0], en[0], hn[0], he[0]);
        if constexpr (PD == 2) {
            issue(kk + 1, un[1], en[1], hn[1], he[1]);
            issue_f(kk, fr[0]);
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

// 2D paired pass (Laplacian): a wavefront marches a strip of 128 nodes of x
// (pairs as in the 3D paired pass, the two outside x-neighbours loaded as one
// extra word per row) along y through a chunk of rows.  y-neighbours are the
// thread's own three-row ring, so there is no LDS and no barrier; the four
// wavefronts of a workgroup take four consecutive chunks of one strip.
template <int PD, bool IR, typename E = float>
struct Pair2D {
    static constexpr int TX = 2 * BX;
    using E2 = typename PairOf<E>::type;
    static constexpr bool H16 = sizeof(E) == 2;
    const MG_GLOBAL double* __restrict__ uin;
    MG_GLOBAL double* __restrict__ uout;
    const MG_GLOBAL E* __restrict__ e;
    const MG_GLOBAL double* __restrict__ f;
    MG_GLOBAL E* __restrict__ r32;
    IRWords<E> wd;
    int n, x0, y0, y1, flags;
    double c;
    int lane;
    unsigned inx;
    bool hin;
    unsigned xp8, xp4, xh8, xh4;
    Dbl2 un[3], fr[3], uo[3];
    E2 en[3];
    double hn[3], ho[3];
    E he[3];
    double acc = 0.0;
    double mxr = 0.0;

    __device__ __forceinline__ void init() {
        const int xa = x0 + 2 * lane;
        inx = (xa <= n - 2 ? 1u : 0u) | (xa + 1 <= n - 2 ? 2u : 0u);
        const unsigned xp = (unsigned)min(xa, n - 2);
        xp8 = xp * 8u;
        xp4 = xp * (unsigned)sizeof(E);
        const int xl = x0 - 1, xr = min(x0 + TX, n - 1);
        const unsigned xh = (unsigned)(lane < 32 ? xl : xr);
        xh8 = xh * 8u;
        xh4 = xh * (unsigned)sizeof(E);
        hin = lane == 0 ? xl >= 1 : (x0 + TX <= n - 2);
    }
    __device__ __forceinline__ void issue(int y, Dbl2& du, E2& de, double& dh, E& dhe) {
        const size_t off = (size_t)min(max(y, 0), n - 1) * n;
        du = ld_d2(uin + off, xp8);
        dh = ld_off(uin + off, xh8);
        if constexpr (IR) {
            if (!(flags & IR_NO_UPDATE)) {
                de = ld_f2(e + off, xp4);
                dhe = ld_off(e + off, xh4);
            } else {
                de = E2{(E)0, (E)0};
                dhe = (E)0;
            }
        }
    }
    __device__ __forceinline__ void issue_f(int y, Dbl2& dst) { dst = ld_d2(f + (size_t)min(max(y, 0), n - 1) * n, xp8); }

    template <int P>
    __device__ __forceinline__ void step(int j) {
        constexpr int S0 = P, S1 = (P + 2) % 3, S2 = (P + 1) % 3, SN = (P + PD) % 3;
        const bool yin = j >= 1 && j <= n - 2;
        Dbl2 v = un[S0];
        double h = hn[S0];
        if constexpr (IR) {
            if (!(flags & IR_NO_UPDATE)) {
                if (yin && (inx & 1u)) v.a = v.a + wd.incr(en[S0].a);
                if (yin && (inx & 2u)) v.b = v.b + wd.incr(en[S0].b);
                if (yin && hin) h = h + wd.incr(he[S0]);
                if (yin && j >= y0 && j < y1) {
                    MG_GLOBAL double* row = uout + (size_t)j * n;
                    if (inx == 3u) st_d2(row, xp8, v);
                    else if (inx & 1u) st_off(row, xp8, v.a);
                }
            }
        }
        uo[S0] = v;
        ho[S0] = h;
        if constexpr (PD == 2) issue_f(j + 1, fr[S2]);
        else issue_f(j, fr[S0]);
        issue(j + PD, un[SN], en[SN], hn[SN], he[SN]);
        const int jj = j - 1;  // residual row
        const Dbl2 uc = uo[S1];
        double wa = lane_prev(uc.b), eb = lane_next(uc.a);  // every lane active
        if (lane == 0) wa = ho[S1];
        if (lane == BX - 1) eb = ho[S1];
        if (jj >= y0) {
            const double ra = res_lap2<double>(uc.a, wa, uc.b, uo[S2].a, uo[S0].a, fr[S1].a, c);
            const double rb = res_lap2<double>(uc.b, uc.a, eb, uo[S2].b, uo[S0].b, fr[S1].b, c);
            if constexpr (IR) {
                MG_GLOBAL E* row = r32 + (size_t)jj * n;
                const E2 rv{wd.res(ra), wd.res(rb)};
                if (inx == 3u) st_f2(row, xp4, rv);
                else if (inx & 1u) st_off(row, xp4, rv.a);
            }
            if (inx & 1u) acc += ra * ra;
            if (inx & 2u) acc += rb * rb;
            if constexpr (H16) {
                if (inx & 1u) mxr = fmax(mxr, fabs(ra));
                if (inx & 2u) mxr = fmax(mxr, fabs(rb));
            }
        }
    }

    __device__ __forceinline__ void run() {
        init();
        if (y0 >= y1) return;  // a wavefront past the last chunk
        int j = y0 - 1;
        const int jend = y1;
        fr[0] = fr[1] = fr[2] = Dbl2{0.0, 0.0};
        uo[1] = uo[2] = Dbl2{0.0, 0.0};
        ho[1] = ho[2] = 0.0;
        issue(j, un[0], en[0], hn[0], he[0]);
        if constexpr (PD == 2) {
            issue(j + 1, un[1], en[1], hn[1], he[1]);
            issue_f(j, fr[0]);
        }
        for (; j + 2 <= jend; j += 3) {
            step<0>(j);
            step<1>(j + 1);
            step<2>(j + 2);
        }
        if (j <= jend) step<0>(j);
        if (j + 1 <= jend) step<1>(j + 1);
    }
};

template <int PD, bool IR, typename E = float>
__device__ __forceinline__ void pair2d_body(const GridDesc* gd, const IRDesc* ird, int sel, int flags,
                                            double* __restrict__ part, int pstride, int ychunk) {
    using S = Pair2D<PD, IR, E>;
    __shared__ double red[4];
    S s;
    int n, inst;
    double* pmax = nullptr;
    if constexpr (IR) {
        const IRDesc d = *ird;
        if (d.par) sel = *gp(d.par);
        n = d.n;
        inst = d.inst;
        s.uin = gp((const double*)(sel ? d.u[1] : d.u[0]));
        s.uout = gp(sel ? d.u[0] : d.u[1]);
        s.e = gp((const E*)d.e);
        s.f = gp(d.f);
        s.r32 = gp((E*)d.r);
        s.c = d.c;
        if constexpr (S::H16) {
            const MG_GLOBAL double* scl = gp(d.scl);
            s.wd.inv = 1.0 / scl[0];
            s.wd.sr = (float)fp16_scale(scl[1]);
            pmax = d.pmax;
        }
    } else {
        const GridDesc d = *gd;
        n = d.n;
        inst = d.inst;
        s.uin = gp((const double*)(sel ? d.t : d.u));
        s.uout = nullptr;
        s.e = nullptr;
        s.f = gp((const double*)d.f);
        s.r32 = nullptr;
        s.c = d.c;
    }
    const int ntx = (n - 2 + S::TX - 1) / S::TX;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int tx = tile % ntx, tb = tile / ntx;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    s.n = n;
    s.x0 = 1 + tx * S::TX;
    s.y0 = min(1 + (tb * 4 + w) * ychunk, n - 1);
    s.y1 = min(s.y0 + ychunk, n - 1);
    s.flags = flags;
    s.lane = threadIdx.x & 63;
    s.run();
    const double t = block_sum_w<4>(s.acc, red);
    if (threadIdx.x == 0) part[(size_t)inst * pstride + blockIdx.x] = t;
    if constexpr (S::H16) {
        const double mx = block_max_w<4>(s.mxr, red);
        if (threadIdx.x == 0) pmax[(size_t)inst * pstride + blockIdx.x] = mx;
    }
}

template <int PD>
__global__ __launch_bounds__(NT) void k_norm2d_p(const GridDesc* __restrict__ descs, int sel,
                                                 double* __restrict__ part, int pstride, int ychunk) {
    const GridDesc* d = descs + blockIdx.y;
    if (d->done && *gp(d->done)) return;
    pair2d_body<PD, false>(d, nullptr, sel, 0, part, pstride, ychunk);
}

template <int PD, int FL, typename E = float>
__global__ __launch_bounds__(NT) void k_ir2d_p(const IRDesc* __restrict__ descs, int sel, double* __restrict__ part,
                                               int pstride, int ychunk) {
    const IRDesc* d = descs + blockIdx.y;
    if (d->done && *gp(d->done)) return;
    pair2d_body<PD, true, E>(nullptr, d, sel, FL, part, pstride, ychunk);
}

template <int BY, int PD, bool IR, int WV, typename E = float>
__device__ __forceinline__ void pair3d_body(const GridDesc* gd, const IRDesc* ird, int sel, int flags,
                                            double* __restrict__ part, int pstride, int zchunk) {
    using S = Pair3D<BY, PD, IR, WV, E>;
    __shared__ double red[WV];
    __shared__ Dbl2 U[3][BY][BX];
    S s;
    int n, inst;
    double* pmax = nullptr;
    if constexpr (IR) {
        const IRDesc d = *ird;
        if (d.par) sel = *gp(d.par);
        n = d.n;
        inst = d.inst;
        s.uin = gp((const double*)(sel ? d.u[1] : d.u[0]));
        s.uout = gp(sel ? d.u[0] : d.u[1]);
        s.e = gp((const E*)d.e);
        s.f = gp(d.f);
        s.r32 = gp((E*)d.r);
        s.c = d.c;
        if constexpr (S::H16) {
            const MG_GLOBAL double* scl = gp(d.scl);
            s.wd.inv = 1.0 / scl[0];
            s.wd.sr = (float)fp16_scale(scl[1]);
            pmax = d.pmax;
        }
    } else {
        const GridDesc d = *gd;
        n = d.n;
        inst = d.inst;
        s.uin = gp((const double*)(sel ? d.t : d.u));
        s.uout = nullptr;
        s.e = nullptr;
        s.f = gp((const double*)d.f);
        s.r32 = nullptr;
        s.c = d.c;
    }
    s.U = U;
    const int ntx = (n - 2 + S::TX - 1) / S::TX, nty = (n - 2 + S::TY - 1) / S::TY;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int tx = tile % ntx, t2 = tile / ntx, ty = t2 % nty, tz = t2 / nty;
    s.n = n;
    s.x0 = 1 + tx * S::TX;
    s.y0 = 1 + ty * S::TY;
    s.z0 = 1 + tz * zchunk;
    s.z1 = min(s.z0 + zchunk, n - 1);
    s.kstart = s.z0 - 1;
    s.kend = s.z1;
    s.flags = flags;
    s.lane = threadIdx.x & 63;
    s.w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    s.run();
    const double t = block_sum_w<WV>(s.acc, red);
    if (threadIdx.x == 0) part[(size_t)inst * pstride + blockIdx.x] = t;
    if constexpr (S::H16) {
        const double mx = block_max_w<WV>(s.mxr, red);
        if (threadIdx.x == 0) pmax[(size_t)inst * pstride + blockIdx.x] = mx;
    }
}

template <int BY, int PD, int WV>
__global__ __launch_bounds__(64 * WV) void k_norm3d_p(const GridDesc* __restrict__ descs, int sel,
                                                      double* __restrict__ part, int pstride, int zchunk) {
    const GridDesc* d = descs + blockIdx.y;
    if (d->done && *gp(d->done)) return;
    pair3d_body<BY, PD, false, WV>(d, nullptr, sel, 0, part, pstride, zchunk);
}

template <int BY, int PD, int FL, int WV, typename E = float>
__global__ __launch_bounds__(64 * WV) void k_ir3d_p(const IRDesc* __restrict__ descs, int sel,
                                                    double* __restrict__ part, int pstride, int zchunk) {
    const IRDesc* d = descs + blockIdx.y;
    if (d->done && *gp(d->done)) return;
    pair3d_body<BY, PD, true, WV, E>(nullptr, d, sel, FL, part, pstride, zchunk);
}

template <bool VAR, int BY, int PD, int WV>
__global__ __launch_bounds__(64 * WV) void k_norm3d(const GridDesc* __restrict__ descs, int sel,
                                                    double* __restrict__ part, int pstride, int zchunk) {
    const GridDesc* d = descs + blockIdx.y;
    if (d->done && *gp(d->done)) return;
    resid3d_body<VAR, BY, PD, false, WV>(d, nullptr, sel, 0, part, pstride, zchunk);
}

// ---------------------------------------------------------------------------
// FP64 refinement pass: u_out = u_in + e (inner), r = f - A u_out (FP64),
// r32 = (float) r on inner nodes, partial sums of r^2.
// ---------------------------------------------------------------------------

template <bool VAR, int BY, int FL>
__global__ __launch_bounds__(NT) void k_ir2d(const IRDesc* __restrict__ descs, int sel, double* __restrict__ part,
                                             int pstride) {
    constexpr int flags = FL;
    const IRDesc d = descs[blockIdx.y];
    __shared__ double red4[4];
    if (d.done && *gp(d.done)) return;
    if (d.par) sel = *gp(d.par);
    constexpr int TX = BX - 2, TY = BY - 2, RPT = BY / 4;
    const int n = d.n;
    const int ntx = (n - 2 + TX - 1) / TX;
    const int tile = blockIdx.x;
    const int x0 = 1 + (tile % ntx) * TX, y0 = 1 + (tile / ntx) * TY;
    const MG_GLOBAL double* __restrict__ uin = gp((const double*)(sel ? d.u[1] : d.u[0]));
    MG_GLOBAL double* __restrict__ uout = gp(sel ? d.u[0] : d.u[1]);
    const MG_GLOBAL float* __restrict__ e = gp((const float*)d.e);
    const MG_GLOBAL double* __restrict__ f = gp(d.f);
    const MG_GLOBAL double* __restrict__ kf = gp(d.k);
    MG_GLOBAL float* __restrict__ r32 = gp((float*)d.r);
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

template <bool VAR, int BY, int PD, int FL, int WV>
__global__ __launch_bounds__(64 * WV) void k_ir3d(const IRDesc* __restrict__ descs, int sel, double* __restrict__ part,
                                                  int pstride, int zchunk) {
    const IRDesc* d = descs + blockIdx.y;
    if (d->done && *gp(d->done)) return;
    resid3d_body<VAR, BY, PD, true, WV>(nullptr, d, sel, FL, part, pstride, zchunk);
}

// Sum of np partials by one workgroup in a fixed order: thread t takes
// elements t, t + NT, t + 2 NT, ... into eight interleaved accumulators (eight
// loads in flight per thread), combined pairwise, then the fixed-order
// workgroup sum.  Result valid in thread 0.
__device__ __forceinline__ double sum_parts(const double* __restrict__ p, int np, double* red4) {
    const MG_GLOBAL double* __restrict__ q = gp(p);
    double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int i = threadIdx.x;
    for (; i + 7 * NT < np; i += 8 * NT) {
#pragma unroll
        for (int j = 0; j < 8; ++j) a[j] += q[i + j * NT];
    }
    for (int j = 0; i < np; i += NT, ++j) a[j] += q[i];  // at most seven more
    const double s = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    return block_sum(s, red4);
}

__global__ __launch_bounds__(NT) void k_norm_finalize(const double* __restrict__ part, int pstride, int nparts,
                                                      int row0, double* __restrict__ norm) {
    __shared__ double red4[4];
    const int row = row0 + blockIdx.x;
    const double t = sum_parts(part + (size_t)row * pstride, nparts, red4);
    if (threadIdx.x == 0) norm[row] = sqrt(t);
}

// Half-precision form: norm as k_norm_finalize (one row), the largest |r| of
// the pass from its partial maxima, and the scale state for the next pass.
__global__ __launch_bounds__(NT) void k_norm_finalize_f16(const double* __restrict__ part,
                                                          const double* __restrict__ pmax, int nparts,
                                                          double* __restrict__ norm, double* __restrict__ scl,
                                                          const int* __restrict__ done) {
    __shared__ double red4[4];
    const double t = sum_parts(part, nparts, red4);
    double m = 0.0;
    for (int i = threadIdx.x; i < nparts; i += NT) m = fmax(m, pmax[i]);
    const double mx = block_max_w<4>(m, red4);
    if (threadIdx.x == 0) {
        norm[0] = sqrt(t);
        if (!(done && *done)) {
            scl[0] = fp16_scale(scl[1]);
            scl[1] = mx;
        }
    }
}

__global__ __launch_bounds__(NT) void k_norm_finalize_rows(const double* __restrict__ part, int pstride,
                                                           const int* __restrict__ nparts,
                                                           const int* __restrict__ rows, double* __restrict__ norm) {
    __shared__ double red4[4];
    const int row = rows[blockIdx.x];
    const double t = sum_parts(part + (size_t)row * pstride, nparts[row], red4);
    if (threadIdx.x == 0) norm[row] = sqrt(t);
}

__global__ void k_set_rows(int* __restrict__ arr, int v, const int* __restrict__ rows, int nrows) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < nrows) arr[rows[j]] = v;
}

__global__ void k_solve_init_rows(const double* __restrict__ norm, double* __restrict__ norm0, int* __restrict__ done,
                                  int* __restrict__ steps, int* __restrict__ status, int* __restrict__ par,
                                  const int* __restrict__ rows, int nrows) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nrows) return;
    const int i = rows[j];
    const double r = norm[i];
    norm0[i] = r;
    steps[i] = 0;
    if (par) par[i] = 0;
    const bool zero = r == 0.0;
    const bool bad = !(r == r) || r > 1e300;
    status[i] = bad ? -5 : (zero ? 0 : 1);
    done[i] = (zero || bad) ? 1 : 0;
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
                            double tol, int max_steps, int ninst, int* __restrict__ par) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ninst || done[i]) return;
    const double r = norm[i], r0 = norm0[i];
    const int s = steps[i] + 1;
    steps[i] = s;
    if (par) par[i] ^= 1;  // the refinement pass of this step wrote the other buffer
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

// Face coefficients of a 3D level: +x, +y, +z face of every node by the
// harmonic mean of its two nodes (1 where the face leaves the grid).
template <typename T>
__global__ __launch_bounds__(NT) void k_faces3d(const T* __restrict__ k, T* __restrict__ fx, int n) {
    const size_t N = (size_t)n * n * n, sz = (size_t)n * n;
    for (size_t p = (size_t)blockIdx.x * NT + threadIdx.x; p < N; p += (size_t)gridDim.x * NT) {
        const int i = (int)(p % n);
        const size_t r = p / n;
        const int j = (int)(r % n);
        const int kz = (int)(r / n);
        const T kp = k[p];
        fx[p] = i < n - 1 ? kface(kp, k[p + 1]) : T(1);
        fx[N + p] = j < n - 1 ? kface(kp, k[p + n]) : T(1);
        fx[2 * N + p] = kz < n - 1 ? kface(kp, k[p + sz]) : T(1);
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

}  // namespace

template <bool VARV, int BY, int PD>
hipError_t launch_norm3d_w(const GridDesc* d, int sel, double* partial, int pstride, TileCfg cfg, dim3 grid,
                           hipStream_t s) {
    if (cfg.xp == 2) {  // two nodes per lane: Laplacian only, at most four rows per thread
        if constexpr (VARV) return hipErrorInvalidValue;
        if (cfg.wv == 8) {
            if constexpr (BY >= 16) {
                k_norm3d_p<BY, PD, 8><<<grid, 512, 0, s>>>(d, sel, partial, pstride, cfg.zchunk);
                return hipSuccess;
            }
            return hipErrorInvalidValue;
        }
        if (cfg.wv != 4) return hipErrorInvalidValue;
        if constexpr (BY <= 16) {
            k_norm3d_p<BY, PD, 4><<<grid, NT, 0, s>>>(d, sel, partial, pstride, cfg.zchunk);
            return hipSuccess;
        }
        return hipErrorInvalidValue;
    }
    if (cfg.wv == 8) {
        if constexpr (BY >= 16) {
            k_norm3d<VARV, BY, PD, 8><<<grid, 512, 0, s>>>(d, sel, partial, pstride, cfg.zchunk);
            return hipSuccess;
        }
        return hipErrorInvalidValue;
    }
    if (cfg.wv != 4) return hipErrorInvalidValue;
    if constexpr (VARV && BY > 16) return hipErrorInvalidValue;
    else k_norm3d<VARV, BY, PD, 4><<<grid, NT, 0, s>>>(d, sel, partial, pstride, cfg.zchunk);
    return hipSuccess;
}

template <bool VARV>
hipError_t launch_norm3d(const GridDesc* d, int sel, double* partial, int pstride, TileCfg cfg, dim3 grid,
                         hipStream_t s) {
    const bool p2 = cfg.pd == 2;
    switch (cfg.by) {
        case 8:
            return p2 ? launch_norm3d_w<VARV, 8, 2>(d, sel, partial, pstride, cfg, grid, s)
                      : launch_norm3d_w<VARV, 8, 1>(d, sel, partial, pstride, cfg, grid, s);
        case 16:
            return p2 ? launch_norm3d_w<VARV, 16, 2>(d, sel, partial, pstride, cfg, grid, s)
                      : launch_norm3d_w<VARV, 16, 1>(d, sel, partial, pstride, cfg, grid, s);
        case 32:
            return p2 ? launch_norm3d_w<VARV, 32, 2>(d, sel, partial, pstride, cfg, grid, s)
                      : launch_norm3d_w<VARV, 32, 1>(d, sel, partial, pstride, cfg, grid, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_norm(int dim, bool var, const GridDesc* d, int ninst, int n, int sel, double* partial, int pstride,
                       TileCfg cfg, hipStream_t s) {
    const dim3 grid(norm_tiles(dim, n, cfg), ninst);
    if ((int)grid.x > pstride) return hipErrorInvalidValue;
    if (dim == 2 && cfg.xp == 2) {  // two nodes per lane, marching along y: Laplacian only
        if (var) return hipErrorInvalidValue;
        if (cfg.pd == 2) k_norm2d_p<2><<<grid, NT, 0, s>>>(d, sel, partial, pstride, cfg.zchunk);
        else k_norm2d_p<1><<<grid, NT, 0, s>>>(d, sel, partial, pstride, cfg.zchunk);
    } else if (dim == 2) {
        if (var) {
            MG_BY_SWITCH(cfg.by, (k_norm2d<true, BY><<<grid, NT, 0, s>>>(d, sel, partial, pstride)))
        } else {
            MG_BY_SWITCH(cfg.by, (k_norm2d<false, BY><<<grid, NT, 0, s>>>(d, sel, partial, pstride)))
        }
    } else {
        const hipError_t e = var ? launch_norm3d<true>(d, sel, partial, pstride, cfg, grid, s)
                                 : launch_norm3d<false>(d, sel, partial, pstride, cfg, grid, s);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

// 3D pass geometries (rows x wavefronts): 8x4, 16x4, 32x4 (at most 16 rows
// with a coefficient field, four rows per thread), 16x8 and 32x8.
template <bool VARV, int FL, int BY, int PD>
hipError_t launch_ir3d_w(const IRDesc* d, int sel, double* partial, int pstride, TileCfg cfg, dim3 grid,
                         hipStream_t s) {
    if (cfg.xp == 2) {  // two nodes per lane: Laplacian only, at most four rows per thread
        if constexpr (VARV) return hipErrorInvalidValue;
        if (cfg.wv == 8) {
            if constexpr (BY >= 16) {
                k_ir3d_p<BY, PD, FL, 8><<<grid, 512, 0, s>>>(d, sel, partial, pstride, cfg.zchunk);
                return hipSuccess;
            }
            return hipErrorInvalidValue;
        }
        if (cfg.wv != 4) return hipErrorInvalidValue;
        if constexpr (BY <= 16) {
            k_ir3d_p<BY, PD, FL, 4><<<grid, NT, 0, s>>>(d, sel, partial, pstride, cfg.zchunk);
            return hipSuccess;
        }
        return hipErrorInvalidValue;
    }
    if (cfg.wv == 8) {
        if constexpr (BY >= 16) {
            k_ir3d<VARV, BY, PD, FL, 8><<<grid, 512, 0, s>>>(d, sel, partial, pstride, cfg.zchunk);
            return hipSuccess;
        }
        return hipErrorInvalidValue;
    }
    if (cfg.wv != 4) return hipErrorInvalidValue;
    if constexpr (VARV && BY > 16) return hipErrorInvalidValue;  // four rows per thread with k
    else k_ir3d<VARV, BY, PD, FL, 4><<<grid, NT, 0, s>>>(d, sel, partial, pstride, cfg.zchunk);
    return hipSuccess;
}

template <bool VARV, int FL>
hipError_t launch_ir_fl(int dim, const IRDesc* d, int sel, double* partial, int pstride, TileCfg cfg, dim3 grid,
                        hipStream_t s) {
    if (dim == 2 && cfg.xp == 2) {  // two nodes per lane, marching along y: Laplacian only
        if constexpr (VARV) return hipErrorInvalidValue;
        if (cfg.pd == 2) k_ir2d_p<2, FL><<<grid, NT, 0, s>>>(d, sel, partial, pstride, cfg.zchunk);
        else k_ir2d_p<1, FL><<<grid, NT, 0, s>>>(d, sel, partial, pstride, cfg.zchunk);
        return hipSuccess;
    }
    if (dim == 2) {
        MG_BY_SWITCH(cfg.by, (k_ir2d<VARV, BY, FL><<<grid, NT, 0, s>>>(d, sel, partial, pstride)))
        return hipSuccess;
    }
    const bool p2 = cfg.pd == 2;
    switch (cfg.by) {
        case 8:
            return p2 ? launch_ir3d_w<VARV, FL, 8, 2>(d, sel, partial, pstride, cfg, grid, s)
                      : launch_ir3d_w<VARV, FL, 8, 1>(d, sel, partial, pstride, cfg, grid, s);
        case 16:
            return p2 ? launch_ir3d_w<VARV, FL, 16, 2>(d, sel, partial, pstride, cfg, grid, s)
                      : launch_ir3d_w<VARV, FL, 16, 1>(d, sel, partial, pstride, cfg, grid, s);
        case 32:
            return p2 ? launch_ir3d_w<VARV, FL, 32, 2>(d, sel, partial, pstride, cfg, grid, s)
                      : launch_ir3d_w<VARV, FL, 32, 1>(d, sel, partial, pstride, cfg, grid, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_ir_update(int dim, bool var, const IRDesc* d, int ninst, int n, int sel, int flags,
                            double* partial, int pstride, TileCfg cfg, hipStream_t s) {
    const dim3 grid(norm_tiles(dim, n, cfg), ninst);
    if ((int)grid.x > pstride) return hipErrorInvalidValue;
    hipError_t e;
    if (flags == IR_NO_UPDATE) {
        e = var ? launch_ir_fl<true, IR_NO_UPDATE>(dim, d, sel, partial, pstride, cfg, grid, s)
                : launch_ir_fl<false, IR_NO_UPDATE>(dim, d, sel, partial, pstride, cfg, grid, s);
    } else if (flags == 0) {
        e = var ? launch_ir_fl<true, 0>(dim, d, sel, partial, pstride, cfg, grid, s)
                : launch_ir_fl<false, 0>(dim, d, sel, partial, pstride, cfg, grid, s);
    } else {
        return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

hipError_t launch_ir_update_f16(int dim, const IRDesc* d, int ninst, int n, int sel, int flags, double* partial,
                                int pstride, TileCfg cfg, hipStream_t s) {
    const dim3 grid(norm_tiles(dim, n, cfg), ninst);
    if ((int)grid.x > pstride || cfg.xp != 2) return hipErrorInvalidValue;
    if (flags != 0 && flags != IR_NO_UPDATE) return hipErrorInvalidValue;
    const bool nu = flags == IR_NO_UPDATE, p2 = cfg.pd == 2;
#define MG_IR16(FLV, PDV)                                                                                     \
    do {                                                                                                      \
        if (dim == 2) {                                                                                       \
            k_ir2d_p<PDV, FLV, half_t><<<grid, NT, 0, s>>>(d, sel, partial, pstride, cfg.zchunk);             \
        } else if (cfg.wv == 8 && cfg.by == 16) {                                                             \
            k_ir3d_p<16, PDV, FLV, 8, half_t><<<grid, 512, 0, s>>>(d, sel, partial, pstride, cfg.zchunk);     \
        } else if (cfg.wv == 8 && cfg.by == 32) {                                                             \
            k_ir3d_p<32, PDV, FLV, 8, half_t><<<grid, 512, 0, s>>>(d, sel, partial, pstride, cfg.zchunk);     \
        } else if (cfg.wv == 4 && cfg.by == 8) {                                                              \
            k_ir3d_p<8, PDV, FLV, 4, half_t><<<grid, NT, 0, s>>>(d, sel, partial, pstride, cfg.zchunk);       \
        } else if (cfg.wv == 4 && cfg.by == 16) {                                                             \
            k_ir3d_p<16, PDV, FLV, 4, half_t><<<grid, NT, 0, s>>>(d, sel, partial, pstride, cfg.zchunk);      \
        } else {                                                                                              \
            return hipErrorInvalidValue;                                                                      \
        }                                                                                                     \
    } while (0)
    if (nu) {
        if (p2) MG_IR16(IR_NO_UPDATE, 2);
        else MG_IR16(IR_NO_UPDATE, 1);
    } else {
        if (p2) MG_IR16(0, 2);
        else MG_IR16(0, 1);
    }
#undef MG_IR16
    return hipGetLastError();
}

hipError_t launch_norm_finalize_f16(const double* partial, const double* pmax, int nparts, double* norm, double* scl,
                                    const int* done, hipStream_t s) {
    k_norm_finalize_f16<<<1, NT, 0, s>>>(partial, pmax, nparts, norm, scl, done);
    return hipGetLastError();
}

hipError_t launch_norm_finalize(const double* partial, int pstride, int nparts, int row0, int ninst, double* norm,
                                hipStream_t s) {
    k_norm_finalize<<<ninst, NT, 0, s>>>(partial, pstride, nparts, row0, norm);
    return hipGetLastError();
}

hipError_t launch_norm_finalize_rows(const double* partial, int pstride, const int* nparts, const int* rows, int nrows,
                                     double* norm, hipStream_t s) {
    if (nrows <= 0) return hipSuccess;
    k_norm_finalize_rows<<<nrows, NT, 0, s>>>(partial, pstride, nparts, rows, norm);
    return hipGetLastError();
}

hipError_t launch_set_rows(int* arr, int v, const int* rows, int nrows, hipStream_t s) {
    if (nrows <= 0) return hipSuccess;
    k_set_rows<<<cdiv(nrows, 256), 256, 0, s>>>(arr, v, rows, nrows);
    return hipGetLastError();
}

hipError_t launch_solve_init_rows(const double* norm, double* norm0, int* done, int* steps, int* status, int* par,
                                  const int* rows, int nrows, hipStream_t s) {
    if (nrows <= 0) return hipSuccess;
    k_solve_init_rows<<<cdiv(nrows, 256), 256, 0, s>>>(norm, norm0, done, steps, status, par, rows, nrows);
    return hipGetLastError();
}

hipError_t launch_solve_init(const double* norm, double* norm0, int* done, int* steps, int* status, double* hist,
                             int hstride, int ninst, hipStream_t s) {
    k_solve_init<<<cdiv(ninst, 256), 256, 0, s>>>(norm, norm0, done, steps, status, hist, hstride, ninst);
    return hipGetLastError();
}

hipError_t launch_stop_test(const double* norm, const double* norm0, int* done, int* steps, int* status, double* hist,
                            int hstride, double tol, int max_steps, int ninst, hipStream_t s, int* par) {
    k_stop_test<<<cdiv(ninst, 256), 256, 0, s>>>(norm, norm0, done, steps, status, hist, hstride, tol, max_steps,
                                                  ninst, par);
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

template <typename T>
hipError_t launch_faces3d(const T* k, T* fx, int n, hipStream_t s) {
    const size_t total = (size_t)n * n * n;
    const int blocks = (int)std::min<size_t>((total + NT - 1) / NT, 8192);
    k_faces3d<T><<<blocks, NT, 0, s>>>(k, fx, n);
    return hipGetLastError();
}
template hipError_t launch_faces3d<double>(const double*, double*, int, hipStream_t);
template hipError_t launch_faces3d<float>(const float*, float*, int, hipStream_t);

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





}  // namespace mg
