// Kernels of stencil d3q15 with f32 population storage.
#define LBM_TU_STENCIL 3
#define LBM_TU_STORE 1
#include "lbm_instantiate.inc"
