// Batched ensemble kernels of stencil d3q19.
#define LBM_TU_STENCIL 1
#include "lbm_batch_instantiate.inc"
