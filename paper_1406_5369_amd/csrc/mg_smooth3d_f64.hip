// 3D smoothing sweeps in FP64.
#define MG_T double
#include "mg_smooth3d.inl"
