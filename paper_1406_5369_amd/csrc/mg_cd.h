// Kernels of the complex-diffusion form (see mg_cd.hip).  Complex arrays are
// (re, im) pairs of doubles, n^dim cells, x fastest.
#pragma once

#include "mg_internal.h"

namespace mg {

// Problem constants: 1/tau, k theta, cos theta, sin theta (as the host
// evaluated them), relaxation weight.
struct CDConst {
    double itau, ktheta, ct, st, omega;
};
// Level constants: n cells per axis, c = 1/h^2 (h = 1/n).
struct CDLevel {
    int n;
    double c;
};
CDLevel cd_level(int n);

hipError_t cd_compute_g(const void* u, void* g, size_t N, CDConst K, hipStream_t s);
// RBGS colour 'colour' in place (uin == uout; red, colour 0, first: it
// stores the pre-sweep g of its cells in g for the black colour) or a Jacobi
// sweep uin -> uout (g unused), one cell per thread, g of the pre-sweep iterate
hipError_t cd_relax(int dim, bool jacobi, const void* uin, void* uout, const void* f, void* g, CDConst K, CDLevel L,
                    int colour, hipStream_t s);
// whether a level takes the tiled sweep (cd_sweep): 2D always, 3D from n = 128
bool cd_tiled(int dim, int n);
// whether cd_sweep takes the FAS correction (uc, uh) on such a level
bool cd_sweep_corrects(int dim, bool jacobi, int n);
// One smoothing sweep uin -> uout (out of place; RBGS both colours, or Jacobi)
// with the diffusivity of uin, in tiles.  With uc and uh (the coarse iterate
// after and before its cycle, level n/2) the sweep starts from uin + P (uc - uh)
// instead (the FAS correction applied to every loaded value; uin unchanged).
hipError_t cd_sweep(int dim, bool jacobi, const void* uin, void* uout, const void* f, CDConst K, CDLevel L,
                    hipStream_t s, const void* uc = nullptr, const void* uh = nullptr);
// uh = R u, rc = R (f - N(u)) with g of u formed on the fly (n >= 2)
hipError_t cd_restrict(int dim, const void* u, const void* f, void* uh, void* rc, CDConst K, CDLevel L,
                       hipStream_t s);
// fc = N_c(uh) + fc (in place), uc = uh, g of uh formed on the fly
hipError_t cd_coarse_rhs(int dim, const void* uh, void* fc, void* uc, CDConst K, CDLevel Lc, hipStream_t s);
hipError_t cd_prolong(int dim, void* u, const void* uc, const void* uh, int n, hipStream_t s);
hipError_t cd_scale(const void* a, void* out, size_t N, double sc, hipStream_t s);
hipError_t cd_apply_op(int dim, const void* u, const void* g, void* out, CDConst K, CDLevel L, hipStream_t s);
int cd_norm_parts(int dim, int n);
// ||f - N(u)|| (g of u formed on the fly) into *norm (device), part: cd_norm_parts doubles
hipError_t cd_norm(int dim, const void* u, const void* f, CDConst K, CDLevel L, double* part, double* norm,
                   hipStream_t s);

}  // namespace mg
