// Kernels of stencil d3q27 with f64 population storage.
#define LBM_TU_STENCIL 2
#define LBM_TU_STORE 0
#include "lbm_instantiate.inc"
