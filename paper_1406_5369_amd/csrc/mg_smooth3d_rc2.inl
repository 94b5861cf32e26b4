// 3D Laplacian: the first two red-black pre-smoothing sweeps of a level whose
// iterate starts at zero, in one launch (included by mg_smooth3d.inl).
#pragma once

namespace mg {
namespace {

// ---------------------------------------------------------------------------
// One wavefront marches a 64 x BY box along z; lane = x position, the thread
// holds all BY rows of its column (y-neighbours in its own registers,
// x-neighbours from the adjacent lanes, z-neighbours from the plane ring), so
// there is no LDS and no barrier.  The four half-sweeps of Algorithm 1's two
// pre-smoothing sweeps from a zero iterate trail each other by one plane:
// step kk (plane kk enters)
//   R1  red nodes of plane kk:      wd f (the relaxation of a zero iterate)
//   B1  black nodes of plane kk-1 from the red values R1 left
//   R2  red nodes of plane kk-2 from the black values B1 left
//   B2  black nodes of plane kk-3 from the red values R2 left; plane kk-3
//       (both colours) is the output
// Each half-sweep needs its predecessor's values on the neighbouring nodes,
// so half-sweep q is valid on the box minus q rings and the output tile is
// the box minus three rings: (64 - 6) x (BY - 6) nodes.  One ring of five
// planes holds every node's latest value: a half-sweep changes one colour of
// one plane, and each reads its neighbours before the half-sweep that would
// change them next (R2 on plane kk-2 reads the black values of kk-1 and kk-3
// that B1 left; B2 on kk-3 reads the red values of kk-4 and kk-2 that R2
// left).  The per-node expressions are those of two separate sweeps (the
// first with every old value zero), stored values rounded to the storage
// type in between, so the output is the same bit for bit.
// ---------------------------------------------------------------------------

template <typename ST, int BY>
struct Sweep2RC {
    using T = arith_t<ST>;
    static constexpr int H = 3;  // output tile: the box minus three rings
    static constexpr int TX = BX - 2 * H, TY = BY - 2 * H;
    static constexpr int R = 5;  // ring of planes kk-4 .. kk

    const MG_GLOBAL ST* __restrict__ f;
    MG_GLOBAL ST* __restrict__ uout;
    int n, x0, y0, z0, z1, kstart, kend;
    T c, wd, om;
    int lane, gx;
    bool coli;
    unsigned xb;
    size_t pl;

    T v[R][BY];   // latest value of every node of planes kk-4 .. kk
    T fr[R][BY];  // f of planes kk-3 .. kk+1 (kk+1 in flight)

    __device__ __forceinline__ int gy(int m) const { return y0 - H + m; }  // wave-uniform
    __device__ __forceinline__ int rowoff(int m) const { return min(max(gy(m), 0), n - 1) * n; }
    __device__ __forceinline__ bool yin(int m) const { return gy(m) >= 1 && gy(m) <= n - 2; }

    // f of every row of plane z (clamped, always in-bounds addresses; only
    // inner nodes use the values)
    __device__ __forceinline__ void issue_f(int z, T (&dst)[BY]) {
        const size_t zoff = (size_t)min(max(z, 0), n - 1) * pl;
#pragma unroll
        for (int m = 0; m < BY; ++m) dst[m] = ld_off(f + zoff + rowoff(m), xb);
    }

    // Half-sweep q (1 B1, 2 R2, 3 B2) of colour col on plane p (slot A),
    // planes below / above in slots B / U: rows q .. BY-1-q, lanes q .. 63-q.
    template <int q>
    __device__ __forceinline__ void half(T (&A)[BY], const T (&Bv)[BY], const T (&Uv)[BY], const T (&F)[BY], int p,
                                         int col) {
        const bool zin = p >= 1 && p <= n - 2;
        const bool ok = zin && coli && lane >= q && lane <= BX - 1 - q;
#pragma unroll
        for (int m = q; m < BY - q; ++m) {
            const T uc = A[m];
            const T uw = lane_prev(uc), ue = lane_next(uc);  // every lane active
            const T r = res_lap3(uc, uw, ue, A[m - 1], A[m + 1], Bv[m], Uv[m], F[m], c);
            const T nv = stored<ST>(relax<T, false>(uc, r, T(0), c, wd, om));
            if (ok && yin(m) && ((gx + gy(m) + p) & 1) == col) A[m] = nv;
        }
    }

    template <int P>
    __device__ __forceinline__ void step(int kk) {
        constexpr int S0 = P, S1 = (P + 4) % R, S2 = (P + 3) % R, S3 = (P + 2) % R, S4 = (P + 1) % R;
        issue_f(kk + 1, fr[S4]);  // slot of plane kk-4, whose f is no longer read
        // R1 on plane kk: the relaxation of a zero iterate at red inner nodes
        {
            const bool zin = kk >= 1 && kk <= n - 2;
            const T zero = T(0);
#pragma unroll
            for (int m = 0; m < BY; ++m) {
                const T r = res_lap3(zero, zero, zero, zero, zero, zero, zero, fr[S0][m], c);
                const T nv = stored<ST>(relax<T, false>(zero, r, zero, c, wd, om));
                v[S0][m] = (zin && coli && yin(m) && ((gx + gy(m) + kk) & 1) == 0) ? nv : zero;
            }
        }
        if (kk - 1 >= z0 - 2) half<1>(v[S1], v[S2], v[S0], fr[S1], kk - 1, 1);
        if (kk - 2 >= z0 - 1) half<2>(v[S2], v[S3], v[S1], fr[S2], kk - 2, 0);
        const int p3 = kk - 3;
        if (p3 >= z0 && p3 < z1) {
            half<3>(v[S3], v[S4], v[S2], fr[S3], p3, 1);
            const bool ok = coli && lane >= H && lane <= BX - 1 - H && p3 >= 1 && p3 <= n - 2;
            MG_GLOBAL ST* __restrict__ out = uout + (size_t)p3 * pl;
#pragma unroll
            for (int m = H; m < BY - H; ++m)
                if (ok && yin(m)) st_off(out + rowoff(m), xb, (ST)v[S3][m]);
        }
    }

    __device__ __forceinline__ void run() {
        pl = (size_t)n * n;
        const int xc = min(max(gx, 0), n - 1);
        xb = (unsigned)xc * (unsigned)sizeof(ST);
        coli = gx >= 1 && gx <= n - 2;
#pragma unroll
        for (int q = 0; q < R; ++q)
#pragma unroll
            for (int m = 0; m < BY; ++m) v[q][m] = fr[q][m] = T(0);
        int kk = kstart;
        issue_f(kk, fr[0]);
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

template <typename ST, int BY>
__global__ __launch_bounds__(64) void k_smooth3d_zg2(const GridDesc* __restrict__ descs, int sel, int zchunk) {
    const GridDesc d = descs[blockIdx.y];
    if (d.done && *gp(d.done)) return;
    using S = Sweep2RC<ST, BY>;
    using T = arith_t<ST>;
    S s;
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
    // the second sweep's output buffer (its input is the first sweep's, which
    // never leaves the registers)
    s.uout = gp((ST*)((sel & 1) ? d.u : d.t));
    s.f = gp((const ST*)d.f);
    s.c = (T)d.c;
    s.wd = (T)d.wd;
    s.om = (T)d.omega;
    s.lane = threadIdx.x;
    s.gx = s.x0 - S::H + s.lane;
    s.run();
}

}  // namespace
}  // namespace mg
