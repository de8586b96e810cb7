// Kernels of stencil d3q19 with f32 population storage.
#define LBM_TU_STENCIL 1
#define LBM_TU_STORE 1
#include "lbm_instantiate.inc"
