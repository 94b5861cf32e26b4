// 3D smoothing sweeps on binary16 fields (float arithmetic).
#define MG_T half_t
#include "mg_smooth3d.inl"
