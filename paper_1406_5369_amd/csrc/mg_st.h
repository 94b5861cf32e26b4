// Kernels of the constant-stencil operator (see mg_st.hip).  Node-based
// grids, n = 2^L + 1 nodes per axis, FP64, x fastest.
#pragma once

#include "mg_internal.h"

namespace mg {

// Constants of one level: n nodes per axis, c = 1/h^2 (h = 1/(n-1)),
// wd = omega h^2 / s0, and the stencil (centre, -x, +x, -y, +y, -z, +z).
struct STConst {
    int n;
    double c, wd;
    double s[7];
};
STConst st_const(int dim, int n, const double* stencil, double omega);

// RBGS colour in place (uin == uout; colour 0 red, 1 black) or one Jacobi
// sweep uin -> uout (inner nodes; uout's boundary is left as it is)
hipError_t st_relax(int dim, bool jacobi, const double* uin, double* uout, const double* f, const STConst& L,
                    int colour, hipStream_t s);
// fc (inner coarse nodes) = full weighting of the residual f - A u
hipError_t st_restrict(int dim, const double* u, const double* f, double* fc, const STConst& L, hipStream_t s);
// u (inner nodes, n per axis) += bi-/trilinear interpolation of ec
hipError_t st_prolong(int dim, double* u, const double* ec, int n, hipStream_t s);
// n = 3: the single unknown u = f / (c s0)
hipError_t st_coarsest(int dim, double* u, const double* f, const STConst& L, hipStream_t s);
// norm[0] = ||f - A u||_2 over inner nodes (part: st_norm_parts doubles)
int st_norm_parts(int dim, int n);
hipError_t st_norm(int dim, const double* u, const double* f, const STConst& L, double* part, double* norm,
                   hipStream_t s);

}  // namespace mg
