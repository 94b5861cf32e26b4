// Device helpers shared by the HIP kernels of the geometric multigrid V-cycle
// for gfx950 (CDNA4).
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
#pragma once

#include "mg_internal.h"

#include <algorithm>

// Pointers read from device-side descriptors are generic to the compiler;
// every kernel converts them to the global address space so loads and stores
// compile to global_* instructions (flat instructions would also count
// against the LDS wait counter and serialise HBM latency with LDS traffic).
#define MG_GLOBAL __attribute__((address_space(1)))

namespace mg {
namespace {

// Storage and arithmetic types.  FP64 and FP32 fields compute in their own
// type; binary16 fields (the half-precision form of the refinement) are
// stored as _Float16 and computed in float, and every value the method stores
// is rounded to binary16 at the point where it would be written, also when a
// fused kernel keeps it in registers (the red half of a sweep, the corrected
// iterate): stored<S>(v) is v rounded to S and read back.
template <typename S>
struct ArithOf {
    using type = S;
};
template <>
struct ArithOf<half_t> {
    using type = float;
};
template <typename S>
using arith_t = typename ArithOf<S>::type;
template <typename S, typename T>
__device__ __forceinline__ T stored(T v) {
    if constexpr (sizeof(S) == sizeof(T)) return v;
    else return (T)(S)v;
}

template <typename T>
__device__ __forceinline__ MG_GLOBAL T* gp(T* p) {
    return (MG_GLOBAL T*)p;
}

// Element at a 32-bit byte offset from a wave-uniform base: the base stays in
// scalar registers and only the offset is per lane, so the access is a global
// load / store with a scalar base address and no per-lane 64-bit address math.
template <typename T>
__device__ __forceinline__ T ld_off(const MG_GLOBAL T* base, unsigned boff) {
    return *(const MG_GLOBAL T*)((const MG_GLOBAL char*)base + boff);
}
template <typename T>
__device__ __forceinline__ void st_off(MG_GLOBAL T* base, unsigned boff, T v) {
    *(MG_GLOBAL T*)((MG_GLOBAL char*)base + boff) = v;
}


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

// 3D variable-coefficient residual from the six face coefficients (each
// kface of the lower and the upper node of its face).
template <typename T>
__device__ __forceinline__ T res_var3f(T uC, T uW, T uE, T uS, T uN, T uB, T uT, T kxW, T kxC, T kyS, T kyC, T kzB,
                                       T kzC, T f, T c, T& dsum) {
    dsum = ((kxW + kxC) + (kyS + kyC)) + (kzB + kzC);
    const T t = ((kxW * uW + kxC * uE) + (kyS * uS + kyC * uN)) + (kzB * uB + kzC * uT);
    return f - c * (dsum * uC - t);
}

template <typename T>
__device__ __forceinline__ T res_var3(T uC, T uW, T uE, T uS, T uN, T uB, T uT, T kC, T kW, T kE, T kS, T kN, T kB,
                                      T kT, T f, T c, T& dsum) {
    return res_var3f(uC, uW, uE, uS, uN, uB, uT, kface(kW, kC), kface(kC, kE), kface(kS, kC), kface(kC, kN),
                     kface(kB, kC), kface(kC, kT), f, c, dsum);
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
template <typename T, typename P>
__device__ __forceinline__ T interp2(P e, int nc, int i, int j) {
    const auto q = e + (size_t)(j >> 1) * nc + (i >> 1);
    const int oi = i & 1, oj = j & 1;
    if (!oi && !oj) return q[0];
    if (oi && !oj) return T(0.5) * (q[0] + q[1]);
    if (!oi && oj) return T(0.5) * (q[0] + q[nc]);
    return T(0.25) * ((q[0] + q[1]) + (q[nc] + q[nc + 1]));
}

// Trilinear interpolation at fine node (i, j, k); the odd axes are taken in
// x, y, z order (s0 first, s1 second, s2 third).
template <typename T, typename P>
__device__ __forceinline__ T interp3(P e, int nc, int i, int j, int k) {
    const size_t sy = (size_t)nc, sz = (size_t)nc * nc;
    const auto q = e + (size_t)(k >> 1) * sz + (size_t)(j >> 1) * sy + (i >> 1);
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

// Tile of block b in a smoothing launch: XCD bands, or linear order when bit 1
// of the kernel's select argument is set (the autotuner's choice).
__device__ __forceinline__ int sweep_tile(int arg, int b, int G) { return (arg & 2) ? b : xcd_tile(b, G); }

// Deterministic workgroup sum of one double per thread (fixed shuffle order,
// then the WV wave partials pairwise in order).  Result valid in thread 0.
template <int WV>
__device__ __forceinline__ double block_sum_w(double v, double* red) {
    static_assert(WV == 4 || WV == 8, "four or eight wavefronts");
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        s = (red[0] + red[1]) + (red[2] + red[3]);
        if constexpr (WV == 8) s = s + ((red[4] + red[5]) + (red[6] + red[7]));
    }
    return s;
}
__device__ __forceinline__ double block_sum(double v, double* red4) { return block_sum_w<4>(v, red4); }

// Neighbours along x from the adjacent lanes of the same wavefront (DPP
// full-wave shifts: lane i reads lane i-1 / i+1).  Lanes 0 and 63 get 0 and
// are never used as centres.  Executed with every lane active.
__device__ __forceinline__ float lane_prev(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xF, 0xF, false));
}
__device__ __forceinline__ float lane_next(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xF, 0xF, false));
}
__device__ __forceinline__ double lane_prev(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), 0x138, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x138, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double lane_next(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), 0x130, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x130, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// 3D residual from explicit neighbour values.
template <typename T, bool VAR>
__device__ __forceinline__ T res3(T uC, T uW, T uE, T uS, T uN, T uB, T uT, T kC, T kW, T kE, T kS, T kN, T kB, T kT,
                                  T f, T c, T& dsum) {
    if constexpr (VAR) {
        return res_var3(uC, uW, uE, uS, uN, uB, uT, kC, kW, kE, kS, kN, kB, kT, f, c, dsum);
    } else {
        dsum = T(0);
        return res_lap3(uC, uW, uE, uS, uN, uB, uT, f, c);
    }
}

inline int cdiv(int a, int b) { return (a + b - 1) / b; }
inline int nzchunks(int m, int zchunk) { return cdiv(m, zchunk); }

}  // namespace

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

// Tile heights 8 and 16 only (kernels whose 32-row variant would exceed the
// architectural register file).
#define MG_BY_SWITCH16(by, CALL) \
    switch (by) {              \
        case 8: {              \
            constexpr int BY = 8; \
            CALL;              \
        } break;               \
        case 16: {             \
            constexpr int BY = 16; \
            CALL;              \
        } break;               \
        default:               \
            return hipErrorInvalidValue; \
    }


}  // namespace mg
