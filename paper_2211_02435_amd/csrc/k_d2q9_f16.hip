// Kernels of stencil d2q9 with f16 population storage.
#define LBM_TU_STENCIL 0
#define LBM_TU_STORE 2
#include "lbm_instantiate.inc"
