// Kernels of the cell-centred Neumann discretisation (see mg_cc.hip).
#pragma once

#include "mg_internal.h"

namespace mg {

// Constants of one cell-centred level: n cells per axis, c = 1/h^2 (h = 1/n),
// wd[m] = omega h^2 / (2d - m) for a cell with m faces on the boundary.
struct CCConst {
    int n;
    double c;
    double wd[4];
};

size_t cc_cells(int dim, int n);
CCConst cc_const(int dim, int n, double omega);
// RBGS colour 'colour' in place (uin == uout) or a Jacobi sweep uin -> uout
hipError_t cc_relax(int dim, bool jacobi, const double* uin, double* uout, const double* f, CCConst L, int colour,
                    hipStream_t s);
// fc (n/2 cells per axis) = average of the children's residuals f - A u
hipError_t cc_restrict(int dim, const double* u, const double* f, double* fc, CCConst L, hipStream_t s);
// u (n cells per axis) += parent value of ec
hipError_t cc_prolong(int dim, double* u, const double* ec, int n, hipStream_t s);
hipError_t cc_fill(double* v, size_t N, double x, hipStream_t s);
// mean[0] = sum of v in the fixed order / cells; work holds cc_work_doubles values
hipError_t cc_mean(int dim, int n, const double* v, double* work, double* mean, hipStream_t s);
hipError_t cc_remove_mean(int dim, int n, double* v, double* work, double* mean, hipStream_t s);
size_t cc_work_doubles(int dim, int n);
// norm[0] = ||f - A u||_2 (partials: cc_norm_parts doubles)
int cc_norm_parts(int dim, int n);
hipError_t cc_norm(int dim, const double* u, const double* f, CCConst L, double* part, double* norm, hipStream_t s);

}  // namespace mg
