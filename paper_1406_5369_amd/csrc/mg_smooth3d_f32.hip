// 3D smoothing sweeps in FP32.
#define MG_T float
#include "mg_smooth3d.inl"
