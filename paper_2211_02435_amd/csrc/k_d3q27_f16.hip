// Kernels of stencil d3q27 with f16 population storage.
#define LBM_TU_STENCIL 2
#define LBM_TU_STORE 2
#include "lbm_instantiate.inc"
