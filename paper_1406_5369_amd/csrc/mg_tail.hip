// Coarse tail of the V-cycle in one launch: every level from a small grid down
// to the coarsest, one workgroup per instance, all fields in LDS.
//
// Below a few thousand nodes a level is far too small to fill the chip, and
// the six launches a level costs per cycle (two pre-sweeps, residual and
// restriction, correction, two post-sweeps) are pure launch latency.  Here the
// whole descending and ascending leg of Algorithm 1 below the tail's finest
// level runs inside one workgroup with barriers between the steps.  The per-
// point arithmetic is the same as in the level kernels (same helpers, same
// operation order), so results are bitwise those of the level-by-level path:
//   * the coarse iterate starts at zero (Algorithm 1), then nu1 sweeps;
//   * RBGS relaxes all red nodes, then all black nodes, in place (a colour's
//     updates read only the other colour); Jacobi relaxes out of place;
//   * r = f - A u on inner nodes, full weighting onto the coarse inner nodes;
//   * the coarsest grid (n = 3) is solved exactly, u = f / diag;
//   * u += P u_coarse on inner nodes, then nu2 sweeps;
//   * the tail's finest iterate is written back to its level's u.
#include "mg_kern.h"

namespace mg {
namespace {

constexpr int TNT = 1024;  // threads per tail workgroup

// Nodes of all levels from edge N down to 3.
__host__ __device__ constexpr int tail_nodes(int dim, int N) {
    int s = 0;
    for (int m = N;; m = (m - 1) / 2 + 1) {
        s += dim == 2 ? m * m : m * m * m;
        if (m == 3) break;
    }
    return s;
}

// One level of the tail inside the workgroup's LDS arrays: its nodes start at
// 'off' in each array (iterate U, right-hand side F, work W, coefficient K).
template <typename T>
struct Lvl {
    int off, n;
    T c, wd, om;
};

template <typename T, int DIM, bool VAR>
__device__ __forceinline__ T tail_res(const T* u, const T* f, const T* k, int n, T c, int p, T& ds) {
    const int sy = n, sz = n * n;
    if constexpr (DIM == 2) {
        if constexpr (VAR) {
            return res_var2(u[p], u[p - 1], u[p + 1], u[p - sy], u[p + sy], k[p], k[p - 1], k[p + 1], k[p - sy],
                            k[p + sy], f[p], c, ds);
        } else {
            ds = T(0);
            return res_lap2(u[p], u[p - 1], u[p + 1], u[p - sy], u[p + sy], f[p], c);
        }
    } else {
        if constexpr (VAR) {
            return res_var3(u[p], u[p - 1], u[p + 1], u[p - sy], u[p + sy], u[p - sz], u[p + sz], k[p], k[p - 1],
                            k[p + 1], k[p - sy], k[p + sy], k[p - sz], k[p + sz], f[p], c, ds);
        } else {
            ds = T(0);
            return res_lap3(u[p], u[p - 1], u[p + 1], u[p - sy], u[p + sy], u[p - sz], u[p + sz], f[p], c);
        }
    }
}

// Inner node q (0-based over the (n-2)^dim inner nodes) -> node index and
// colour (i + j [+ k]) mod 2.
template <int DIM>
__device__ __forceinline__ int tail_node(int q, int n, int& colour) {
    const int m = n - 2;
    const int i = 1 + q % m;
    const int r = q / m;
    const int j = 1 + (DIM == 2 ? r : r % m);
    const int k = DIM == 2 ? 0 : 1 + r / m;
    colour = (i + j + k) & 1;
    return (k * n + j) * n + i;
}

template <int DIM>
__device__ __forceinline__ int tail_inner(int n) {
    return DIM == 2 ? (n - 2) * (n - 2) : (n - 2) * (n - 2) * (n - 2);
}

// One smoothing sweep of a level (arrays already offset to the level).  The
// LDS arrays hold arithmetic-type values; every iterate value is rounded to
// the storage type ST where the level kernels would store it.  RBGS relaxes
// colour 'first' (0 red, 1 black), then the other one.
template <typename ST, typename T, int DIM, int SM, bool VAR>
__device__ void tail_sweep(T* u, const T* f, T* w, const T* k, const Lvl<T>& L, int first = 0) {
    const int cnt = tail_inner<DIM>(L.n);
    if constexpr (SM == SM_RBGS) {
        for (int half = 0; half < 2; ++half) {
            const int colour = half ^ first;
            for (int q = threadIdx.x; q < cnt; q += TNT) {
                int cl;
                const int p = tail_node<DIM>(q, L.n, cl);
                if (cl != colour) continue;
                T ds;
                const T r = tail_res<T, DIM, VAR>(u, f, k, L.n, L.c, p, ds);
                u[p] = stored<ST>(relax<T, VAR>(u[p], r, ds, L.c, L.wd, L.om));
            }
            __syncthreads();
        }
    } else {
        for (int q = threadIdx.x; q < cnt; q += TNT) {
            int cl;
            const int p = tail_node<DIM>(q, L.n, cl);
            T ds;
            const T r = tail_res<T, DIM, VAR>(u, f, k, L.n, L.c, p, ds);
            w[p] = stored<ST>(relax<T, VAR>(u[p], r, ds, L.c, L.wd, L.om));
        }
        __syncthreads();
        for (int q = threadIdx.x; q < cnt; q += TNT) {
            int cl;
            const int p = tail_node<DIM>(q, L.n, cl);
            u[p] = w[p];
        }
        __syncthreads();
    }
}

// Full weighting of the residual array R (edge nf) around fine node fp; same
// operation order as the restriction kernel.
template <typename T, int DIM>
__device__ __forceinline__ T tail_fw(const T* R, int nf, int fp) {
    const int sy = nf, sz = nf * nf;
    if constexpr (DIM == 2) {
        const T edges = (R[fp - 1] + R[fp + 1]) + (R[fp - sy] + R[fp + sy]);
        const T corners = (R[fp - sy - 1] + R[fp - sy + 1]) + (R[fp + sy - 1] + R[fp + sy + 1]);
        return (T(0.25) * R[fp] + T(0.125) * edges) + T(0.0625) * corners;
    } else {
        const T* Rb = R - sz;
        const T* Ra = R + sz;
        const T faces = ((R[fp - 1] + R[fp + 1]) + (R[fp - sy] + R[fp + sy])) + (Rb[fp] + Ra[fp]);
        const T exy = (R[fp - sy - 1] + R[fp - sy + 1]) + (R[fp + sy - 1] + R[fp + sy + 1]);
        const T exz = (Rb[fp - 1] + Rb[fp + 1]) + (Ra[fp - 1] + Ra[fp + 1]);
        const T eyz = (Rb[fp - sy] + Rb[fp + sy]) + (Ra[fp - sy] + Ra[fp + sy]);
        const T edges = (exy + exz) + eyz;
        const T cz0 = (Rb[fp - sy - 1] + Rb[fp - sy + 1]) + (Rb[fp + sy - 1] + Rb[fp + sy + 1]);
        const T cz1 = (Ra[fp - sy - 1] + Ra[fp - sy + 1]) + (Ra[fp + sy - 1] + Ra[fp + sy + 1]);
        const T corners = cz0 + cz1;
        return ((T(0.125) * R[fp] + T(0.0625) * faces) + T(0.03125) * edges) + T(0.015625) * corners;
    }
}

template <typename ST, int DIM, int SM, bool VAR, int NMAX>
__global__ __launch_bounds__(TNT) void k_tail(const TailDesc* __restrict__ descs, int nu1, int nu2, int post_first) {
    using T = arith_t<ST>;
    constexpr int TOT = tail_nodes(DIM, NMAX);
    __shared__ T Us[TOT];
    __shared__ T Fs[TOT];
    __shared__ T Ws[TOT];
    __shared__ T Ks[VAR ? TOT : 1];
    __shared__ Lvl<T> L[kMaxTailLevels];
    __shared__ int s_tot;
    const TailDesc& td = descs[blockIdx.x];
    const int nl = td.nlev;
    const int* done = td.lv[0].done;
    if (done && *gp(done)) return;
    if (threadIdx.x == 0) {
        int off = 0;
        for (int j = 0; j < nl; ++j) {
            const GridDesc& g = td.lv[j];
            L[j].off = off;
            L[j].n = g.n;
            L[j].c = (T)g.c;
            L[j].wd = (T)g.wd;
            L[j].om = (T)g.omega;
            off += DIM == 2 ? g.n * g.n : g.n * g.n * g.n;
        }
        s_tot = off;
    }
    __syncthreads();
    const int tot = s_tot;
    // every iterate starts at zero; f of the tail's finest level and the
    // coefficients of all levels come from device memory
    const int n0 = td.lv[0].n;
    const int np0 = DIM == 2 ? n0 * n0 : n0 * n0 * n0;
    const MG_GLOBAL ST* __restrict__ f0 = gp((const ST*)td.lv[0].f);
    for (int p = threadIdx.x; p < tot; p += TNT) {
        Us[p] = T(0);
        Ws[p] = T(0);
        Fs[p] = p < np0 ? (T)f0[p] : T(0);
    }
    if constexpr (VAR) {
        for (int j = 0; j < nl; ++j) {
            const MG_GLOBAL T* __restrict__ kg = gp((const T*)td.lv[j].k);
            const int n = L[j].n, np = DIM == 2 ? n * n : n * n * n;
            for (int p = threadIdx.x; p < np; p += TNT) Ks[L[j].off + p] = kg[p];
        }
    }
    __syncthreads();

    // descending leg
    for (int j = 0; j + 1 < nl; ++j) {
        const Lvl<T> lv = L[j];
        T* u = Us + lv.off;
        T* w = Ws + lv.off;
        const T* f = Fs + lv.off;
        const T* k = Ks + (VAR ? lv.off : 0);
        for (int s = 0; s < nu1; ++s) tail_sweep<ST, T, DIM, SM, VAR>(u, f, w, k, lv);
        const int cnt = tail_inner<DIM>(lv.n);
        for (int q = threadIdx.x; q < cnt; q += TNT) {
            int cl;
            const int p = tail_node<DIM>(q, lv.n, cl);
            T ds;
            w[p] = tail_res<T, DIM, VAR>(u, f, k, lv.n, lv.c, p, ds);
        }
        __syncthreads();
        const int nf = lv.n, nc = L[j + 1].n;
        T* fc = Fs + L[j + 1].off;
        const int cc = tail_inner<DIM>(nc);
        for (int q = threadIdx.x; q < cc; q += TNT) {
            int cl;
            const int P = tail_node<DIM>(q, nc, cl);
            const int I = P % nc, J = (P / nc) % nc, K = DIM == 2 ? 0 : P / (nc * nc);
            fc[P] = stored<ST>(tail_fw<T, DIM>(w, nf, ((2 * K) * nf + 2 * J) * nf + 2 * I));
        }
        __syncthreads();
    }
    // coarsest grid: one unknown, u = f / diag
    if (threadIdx.x == 0) {
        const Lvl<T> lv = L[nl - 1];
        const int p = DIM == 2 ? 4 : 13;
        T diag;
        if constexpr (VAR) {
            const T* k = Ks + lv.off;
            const T kC = k[p];
            const T kxW = kface(k[p - 1], kC), kxC = kface(kC, k[p + 1]);
            const T kyS = kface(k[p - 3], kC), kyC = kface(kC, k[p + 3]);
            T dsum;
            if constexpr (DIM == 2) {
                dsum = (kxW + kxC) + (kyS + kyC);
            } else {
                const T kzB = kface(k[p - 9], kC), kzC = kface(kC, k[p + 9]);
                dsum = ((kxW + kxC) + (kyS + kyC)) + (kzB + kzC);
            }
            diag = lv.c * dsum;
        } else {
            diag = lv.c * (DIM == 2 ? T(4) : T(6));
        }
        Us[lv.off + p] = stored<ST>(Fs[lv.off + p] / diag);
    }
    __syncthreads();
    // ascending leg
    for (int j = nl - 2; j >= 0; --j) {
        const Lvl<T> lv = L[j];
        T* u = Us + lv.off;
        T* w = Ws + lv.off;
        const T* f = Fs + lv.off;
        const T* k = Ks + (VAR ? lv.off : 0);
        const T* uc = Us + L[j + 1].off;
        const int nc = L[j + 1].n, n = lv.n;
        const int cnt = tail_inner<DIM>(n);
        for (int q = threadIdx.x; q < cnt; q += TNT) {
            int cl;
            const int p = tail_node<DIM>(q, n, cl);
            const int i = p % n, jj = (p / n) % n, kk = DIM == 2 ? 0 : p / (n * n);
            const T corr = DIM == 2 ? interp2<T>(uc, nc, i, jj) : interp3<T>(uc, nc, i, jj, kk);
            u[p] = stored<ST>(u[p] + corr);
        }
        __syncthreads();
        for (int s = 0; s < nu2; ++s) tail_sweep<ST, T, DIM, SM, VAR>(u, f, w, k, lv, post_first);
    }
    // the tail's finest iterate back to device memory (inner nodes; its
    // boundary there is zero already)
    MG_GLOBAL ST* __restrict__ u0 = gp((ST*)td.lv[0].u);
    const int cnt = tail_inner<DIM>(n0);
    for (int q = threadIdx.x; q < cnt; q += TNT) {
        int cl;
        const int p = tail_node<DIM>(q, n0, cl);
        u0[p] = (ST)Us[p];
    }
}

// ---------------------------------------------------------------------------
// Conjugate gradients on a coarsest level with more than one unknown
// (Algorithm 1: the coarsest grid is solved by a direct solver or by CG), one
// workgroup per instance, every vector in LDS.  From u = 0: r = p = f on the
// inner nodes, then a fixed number of steps (fewer only if r or p^T A p
// becomes zero): q = A p, alpha = (r^T r) / (p^T q), u += alpha p,
// r -= alpha q, beta = (r_new^T r_new) / (r^T r), p = r + beta p.  Inner
// products are formed in FP64 from the vectors' values, each x-row summed
// left to right and the row sums added in row order; alpha and beta are the
// FP64 quotients rounded to the arithmetic type; the vector updates are in
// the arithmetic type and every stored vector value is rounded to the
// storage type ST.
// ---------------------------------------------------------------------------

template <typename T, int DIM, bool VAR>
__device__ __forceinline__ T cg_apply(const T* v, const T* k, int n, T c, int p) {
    const int sy = n, sz = n * n;
    if constexpr (VAR) {
        const T kp = k[p];
        const T kxW = kface(k[p - 1], kp), kxC = kface(kp, k[p + 1]);
        const T kyS = kface(k[p - sy], kp), kyC = kface(kp, k[p + sy]);
        if constexpr (DIM == 2) {
            const T dsum = (kxW + kxC) + (kyS + kyC);
            const T t = (kxW * v[p - 1] + kxC * v[p + 1]) + (kyS * v[p - sy] + kyC * v[p + sy]);
            return c * (dsum * v[p] - t);
        } else {
            const T kzB = kface(k[p - sz], kp), kzC = kface(kp, k[p + sz]);
            const T dsum = ((kxW + kxC) + (kyS + kyC)) + (kzB + kzC);
            const T t = ((kxW * v[p - 1] + kxC * v[p + 1]) + (kyS * v[p - sy] + kyC * v[p + sy])) +
                        (kzB * v[p - sz] + kzC * v[p + sz]);
            return c * (dsum * v[p] - t);
        }
    } else if constexpr (DIM == 2) {
        const T s = (v[p - 1] + v[p + 1]) + (v[p - sy] + v[p + sy]);
        return c * (T(4) * v[p] - s);
    } else {
        const T s = ((v[p - 1] + v[p + 1]) + (v[p - sy] + v[p + sy])) + (v[p - sz] + v[p + sz]);
        return c * (T(6) * v[p] - s);
    }
}

// FP64 inner product over the inner nodes: thread t sums inner row t (x from
// 1 to n-2), thread 0 adds the row sums in order.  Result in every thread.
template <typename T, int DIM>
__device__ __forceinline__ double cg_dot(const T* a, const T* b, int n, double* rows, double* bc) {
    const int m = n - 2;
    const int nrows = DIM == 2 ? m : m * m;
    for (int t = threadIdx.x; t < nrows; t += TNT) {
        const int j = 1 + t % m, k = DIM == 2 ? 0 : 1 + t / m;
        const int base = (k * n + j) * n;
        double s = 0.0;
        for (int i = 1; i <= m; ++i) s += (double)a[base + i] * (double)b[base + i];
        rows[t] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int t = 0; t < nrows; ++t) s += rows[t];
        *bc = s;
    }
    __syncthreads();
    const double v = *bc;
    __syncthreads();  // bc and rows are written again by the next product
    return v;
}

template <typename ST, int DIM, bool VAR, int NMAX>
__global__ __launch_bounds__(TNT) void k_cg(const GridDesc* __restrict__ descs, int iters) {
    using T = arith_t<ST>;
    constexpr int TOT = DIM == 2 ? NMAX * NMAX : NMAX * NMAX * NMAX;
    constexpr int NROWS = DIM == 2 ? NMAX : NMAX * NMAX;
    __shared__ T U[TOT], R[TOT], Pv[TOT], Q[TOT];
    __shared__ T K[VAR ? TOT : 1];
    __shared__ double rows[NROWS];
    __shared__ double bc;
    const GridDesc d = descs[blockIdx.x];
    if (d.done && *gp(d.done)) return;
    const int n = d.n;
    const int np = DIM == 2 ? n * n : n * n * n;
    const T c = (T)d.c;
    const MG_GLOBAL ST* __restrict__ f = gp((const ST*)d.f);
    const int cnt = tail_inner<DIM>(n);
    for (int p = threadIdx.x; p < np; p += TNT) {
        U[p] = T(0);
        R[p] = T(0);
        Pv[p] = T(0);
        Q[p] = T(0);
        if constexpr (VAR) K[p] = gp((const T*)d.k)[p];
    }
    __syncthreads();
    for (int q = threadIdx.x; q < cnt; q += TNT) {
        int cl;
        const int p = tail_node<DIM>(q, n, cl);
        R[p] = (T)f[p];
        Pv[p] = (T)f[p];
    }
    __syncthreads();
    double rr = cg_dot<T, DIM>(R, R, n, rows, &bc);
    for (int it = 0; it < iters && rr > 0.0; ++it) {
        for (int q = threadIdx.x; q < cnt; q += TNT) {
            int cl;
            const int p = tail_node<DIM>(q, n, cl);
            Q[p] = stored<ST>(cg_apply<T, DIM, VAR>(Pv, K, n, c, p));
        }
        __syncthreads();
        const double pq = cg_dot<T, DIM>(Pv, Q, n, rows, &bc);
        if (!(pq > 0.0)) break;
        const T alpha = (T)(rr / pq);
        for (int q = threadIdx.x; q < cnt; q += TNT) {
            int cl;
            const int p = tail_node<DIM>(q, n, cl);
            U[p] = stored<ST>(U[p] + alpha * Pv[p]);
            R[p] = stored<ST>(R[p] - alpha * Q[p]);
        }
        __syncthreads();
        const double rr_new = cg_dot<T, DIM>(R, R, n, rows, &bc);
        const T beta = (T)(rr_new / rr);
        for (int q = threadIdx.x; q < cnt; q += TNT) {
            int cl;
            const int p = tail_node<DIM>(q, n, cl);
            Pv[p] = stored<ST>(R[p] + beta * Pv[p]);
        }
        __syncthreads();
        rr = rr_new;
    }
    MG_GLOBAL ST* __restrict__ u = gp((ST*)d.u);
    for (int p = threadIdx.x; p < np; p += TNT) u[p] = (ST)U[p];
}

}  // namespace

// The tail's LDS holds arithmetic-type values: 4 bytes for FP32 and binary16
// fields, 8 for FP64.
int tail_max_edge(int dim, int elem) {
    if (dim == 2) return elem <= 4 ? 65 : 33;
    return elem <= 4 ? 17 : 9;
}

template <typename T>
hipError_t launch_tail(int dim, int sm, bool var, const TailDesc* d, int ninst, int nu1, int nu2, int post_first,
                       hipStream_t s) {
    if (ninst <= 0) return hipSuccess;
    constexpr bool F = sizeof(arith_t<T>) == 4;
#define MG_TAIL(DIMV, NMAXV)                                                                                     \
    do {                                                                                                      \
        if (sm == SM_RBGS) {                                                                                  \
            if (var) k_tail<T, DIMV, SM_RBGS, true, NMAXV><<<ninst, TNT, 0, s>>>(d, nu1, nu2, post_first);               \
            else k_tail<T, DIMV, SM_RBGS, false, NMAXV><<<ninst, TNT, 0, s>>>(d, nu1, nu2, post_first);                  \
        } else {                                                                                              \
            if (var) k_tail<T, DIMV, SM_JACOBI, true, NMAXV><<<ninst, TNT, 0, s>>>(d, nu1, nu2, post_first);             \
            else k_tail<T, DIMV, SM_JACOBI, false, NMAXV><<<ninst, TNT, 0, s>>>(d, nu1, nu2, post_first);                \
        }                                                                                                     \
    } while (0)
    if constexpr (sizeof(T) == 2) {  // binary16 storage: Laplacian only
        if (var) return hipErrorInvalidValue;
        if (dim == 2) {
            if (sm == SM_RBGS) k_tail<T, 2, SM_RBGS, false, 65><<<ninst, TNT, 0, s>>>(d, nu1, nu2, post_first);
            else k_tail<T, 2, SM_JACOBI, false, 65><<<ninst, TNT, 0, s>>>(d, nu1, nu2, post_first);
        } else {
            if (sm == SM_RBGS) k_tail<T, 3, SM_RBGS, false, 17><<<ninst, TNT, 0, s>>>(d, nu1, nu2, post_first);
            else k_tail<T, 3, SM_JACOBI, false, 17><<<ninst, TNT, 0, s>>>(d, nu1, nu2, post_first);
        }
        return hipGetLastError();
    }
    if (dim == 2) MG_TAIL(2, (F ? 65 : 33));
    else MG_TAIL(3, (F ? 17 : 9));
#undef MG_TAIL
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cg(int dim, bool var, const GridDesc* d, int ninst, int n, int iters, hipStream_t s) {
    const bool f = sizeof(arith_t<T>) == 4;
    if (ninst <= 0) return hipSuccess;
    if (n > tail_max_edge(dim, f ? 4 : 8) || n < 3 || iters < 0) return hipErrorInvalidValue;
    if constexpr (sizeof(T) == 2) {
        if (var) return hipErrorInvalidValue;
        if (dim == 2) k_cg<T, 2, false, 65><<<ninst, TNT, 0, s>>>(d, iters);
        else k_cg<T, 3, false, 17><<<ninst, TNT, 0, s>>>(d, iters);
    } else if constexpr (sizeof(T) == 4) {
        if (dim == 2) {
            if (var) k_cg<T, 2, true, 65><<<ninst, TNT, 0, s>>>(d, iters);
            else k_cg<T, 2, false, 65><<<ninst, TNT, 0, s>>>(d, iters);
        } else {
            if (var) k_cg<T, 3, true, 17><<<ninst, TNT, 0, s>>>(d, iters);
            else k_cg<T, 3, false, 17><<<ninst, TNT, 0, s>>>(d, iters);
        }
    } else {
        if (dim == 2) {
            if (var) k_cg<T, 2, true, 33><<<ninst, TNT, 0, s>>>(d, iters);
            else k_cg<T, 2, false, 33><<<ninst, TNT, 0, s>>>(d, iters);
        } else {
            if (var) k_cg<T, 3, true, 9><<<ninst, TNT, 0, s>>>(d, iters);
            else k_cg<T, 3, false, 9><<<ninst, TNT, 0, s>>>(d, iters);
        }
    }
    return hipGetLastError();
}

template hipError_t launch_cg<double>(int, bool, const GridDesc*, int, int, int, hipStream_t);
template hipError_t launch_cg<float>(int, bool, const GridDesc*, int, int, int, hipStream_t);
template hipError_t launch_cg<half_t>(int, bool, const GridDesc*, int, int, int, hipStream_t);
template hipError_t launch_tail<double>(int, int, bool, const TailDesc*, int, int, int, int, hipStream_t);
template hipError_t launch_tail<float>(int, int, bool, const TailDesc*, int, int, int, int, hipStream_t);
template hipError_t launch_tail<half_t>(int, int, bool, const TailDesc*, int, int, int, int, hipStream_t);

}  // namespace mg
